/*
 * fts.h - C ABI of the fast tensor-product Schwarz smoother library (libfts.so)
 *
 * Additive Schwarz smoothing for the symmetric interior penalty (SIPG) DG
 * discretisation of the Laplacian on Cartesian Q_k meshes, with local solvers
 * by fast diagonalisation, a matrix-free SIPG operator and a geometric
 * multigrid V-cycle (Witte, Arndt, Kanschat, "Fast tensor product Schwarz
 * smoothers for high-order discontinuous Galerkin methods").  All compute runs
 * in HIP kernels for gfx950.
 *
 * Conventions
 *   Vectors   FP64, device memory owned by the caller, contiguous, cell-major:
 *             cells lexicographic with x fastest, and inside a cell the
 *             (k+1)^d DoFs lexicographic with x fastest (Sec. 3, eq. multiindex).
 *             Coefficients are Lagrange values in the Gauss-Lobatto points of
 *             each cell (Sec. 2.1); the inner product is the Euclidean one of the
 *             coefficient space (Sec. 2.1).
 *   Streams   every device call is asynchronous on the given stream (a
 *             hipStream_t passed as void*; NULL = default stream).  No call
 *             synchronises the device unless documented.
 *   Ownership all device memory comes from the caller: vectors and workspaces
 *             are passed in, and the tables of the handles (1-D matrices,
 *             eigenvectors, level vectors, staging buffers, coarse factors,
 *             batch queues, and the BLAS workspace of the coarse setup) are
 *             obtained at creation from the allocator registered with
 *             fts_set_allocator (the Python binding registers torch's
 *             caching allocator); the library never calls hipMalloc.
 *             Handles (fts_level, fts_eigs, fts_hierarchy, fts_batch,
 *             fts_mapped_level) return their memory to that allocator in
 *             *_destroy, which accepts NULL.  Hot calls (apply, residual,
 *             smooth, vcycle, transfers) never allocate.
 *   Errors    every function returns fts_status (0 = FTS_OK, < 0 error); the
 *             last error message of the calling thread is available through
 *             fts_last_error.  No exception crosses the ABI, nothing aborts.
 *             Creation calls validate all arguments; hot calls check handles
 *             and pointers for NULL and report kernel launch failures as
 *             FTS_E_HIP.  Faults of earlier asynchronous work surface at the
 *             next synchronising call as FTS_E_HIP.
 */
#ifndef FTS_H
#define FTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fts_status;
#define FTS_OK 0
#define FTS_E_INVAL (-1)       /* invalid argument */
#define FTS_E_HIP (-2)         /* HIP runtime or kernel launch failure */
#define FTS_E_NOT_SPD (-3)     /* a 1-D mass or operator matrix is not positive definite */
#define FTS_E_UNSUPPORTED (-4) /* dimension / degree / precision not built */
#define FTS_E_SIZE (-5)        /* workspace too small or size overflow */

/* Subdomains of the Schwarz smoother (Sec. 2.3): single cells, or the 2^d
 * cells around each interior vertex. */
typedef enum { FTS_CELL = 0, FTS_VERTEX_PATCH = 1 } fts_patch_kind;

/* Arithmetic of the local-solver contractions (gather, forward transform,
 * eigenvalue scaling, backward transform).  Residual, 1-D setup, transfers
 * and coarse solve are FP64 in every mode; the update of x is accumulated in
 * FP64.  BF16/F16 run the contractions on MFMA with FP32 accumulation. */
typedef enum { FTS_PREC_F64 = 0, FTS_PREC_F32 = 1, FTS_PREC_BF16 = 2, FTS_PREC_F16 = 3 } fts_prec;

/* Rectilinear Cartesian mesh of [0, sum h_x] x [0, sum h_y] (x [0, sum h_z])
 * (Sec. 2.1).  h[a] points to ncells[a] positive widths in HOST memory (read
 * during the call only).  penalty_factor is gamma_hat of eq. (penalty):
 * gamma_e = gamma_hat k (k+1) (1/h+ + 1/h-), h+ = h- on the boundary.
 * Homogeneous Dirichlet conditions are imposed weakly on the whole boundary. */
typedef struct fts_mesh_desc {
    int32_t dim;            /* 2 or 3 */
    int32_t degree;         /* k: 1..9 in 3-D, 1..15 in 2-D */
    int32_t ncells[3];      /* cells per axis (ncells[2] ignored for dim 2) */
    const double *h[3];     /* host arrays of widths */
    double penalty_factor;  /* gamma_hat > 0 */
} fts_mesh_desc;

typedef struct fts_level fts_level;         /* one mesh with its operator tables */
typedef struct fts_eigs fts_eigs;           /* 1-D eigenpairs of all subdomains of a level */
typedef struct fts_hierarchy fts_hierarchy; /* multigrid hierarchy with coarse LU */

/* Device memory allocator of the library: alloc(bytes, ctx) returns device
 * memory of the current device (aligned to 256 bytes, NULL on failure),
 * release(ptr, ctx) takes it back.  Every device allocation of the library
 * goes through it (at handle creation only); with none registered, handle
 * creation fails with FTS_E_HIP.  Register before creating handles and keep
 * it until they are destroyed (their memory is returned to the allocator
 * registered at that time).  Both functions NULL unregisters. */
typedef void *(*fts_alloc_fn)(size_t bytes, void *ctx);
typedef void (*fts_free_fn)(void *ptr, void *ctx);
fts_status fts_set_allocator(fts_alloc_fn alloc, fts_free_fn release, void *ctx);

/* Library version string (static storage). */
const char *fts_version(void);

/* Copies the calling thread's last error message into buf (NUL terminated,
 * truncated to len).  Returns FTS_OK. */
fts_status fts_last_error(char *buf, size_t len);

/* ---- a level: mesh + operator tables ---------------------------------- */

/* Builds the FP64 1-D operator tables of the SIPG form on this mesh (Sec. 3.2,
 * eq. 1Dstiffnessmass, 1Dnitsche, 1Dsipg, 1DsipgVP) and uploads them to the
 * current device.  Validates: dim in {2,3}, 1 <= degree <= 9 (3-D) or 15 (2-D), ncells >= 1,
 * h > 0 and finite, penalty_factor > 0.  *out receives the handle. */
fts_status fts_level_create(const fts_mesh_desc *mesh, fts_level **out);
fts_status fts_level_destroy(fts_level *level);
/* Number of DoFs, (k+1)^d prod ncells; -1 for NULL. */
int64_t fts_level_ndofs(const fts_level *level);

/* ---- a1-a3: 1-D generalised eigenproblems ------------------------------ */

/* For every axis and every subdomain position along it, assembles the 1-D
 * matrices A and M of the subdomain (a cell: eq. 1Dsipg; a vertex patch: the
 * 2x2 block form eq. 1DsipgVP, whose outer faces see the outside neighbours'
 * widths) and solves A S = M S diag(lambda) with S^T M S = I (eq.
 * generalizedEVP) in FP64 on the host (Cholesky + cyclic Jacobi), then
 * uploads S (n x n, row-major, column m = eigenvector m) and lambda (n) per
 * (axis, position), n = k+1 for cells and 2(k+1) for patches.  Positions
 * with bit-identical widths around them share one uploaded table; at a
 * position whose 1-D problem is mirror symmetric (n even) the uploaded modes
 * are reordered, even eigenvectors first, and made exactly even or odd (the
 * local solve is the same operator; fts_eigs_get returns the solver's own
 * order).  Vertex
 * patches need at least 2 cells per axis.  FTS_E_NOT_SPD if M or A is not
 * positive definite (e.g. too small a penalty).  *out receives the handle,
 * valid while the level lives. */
fts_status fts_setup_1d_eigs(const fts_level *level, fts_patch_kind kind, fts_eigs **out);
fts_status fts_eigs_destroy(fts_eigs *eigs);

/* Host copies of the 1-D data of subdomain position `index` along `axis`
 * (0 <= index < ncells[axis] for cells, < ncells[axis]-1 for patches):
 * A, M, S as n x n row-major (any pointer may be NULL), lambda of length n. */
fts_status fts_eigs_get(const fts_eigs *eigs, int32_t axis, int32_t index, double *A, double *M,
                        double *S, double *lambda);
/* n of the subdomains (k+1 or 2(k+1)). */
int32_t fts_eigs_n(const fts_eigs *eigs);

/* How overlapping vertex patches are summed (both give the additive operator
 * of eq. additiveschwarz; they differ only in rounding order):
 *   FTS_SCHEDULE_STAGED  one launch over all patches writes each
 *        patch's correction to a staging buffer owned by the eigs handle
 *        (2^d (k+1)^d doubles per patch, allocated by fts_setup_1d_eigs);
 *        a second launch adds, per cell, the corrections of its 2^d patches
 *        in a fixed order.  Deterministic.  Calls using one eigs handle must
 *        be ordered on one stream (they share the staging buffer).
 *   FTS_SCHEDULE_COLORED 2^d launches, one per parquet color (patches of one
 *        color share no cell, Sec. 2.3), each adding into x directly.
 *   FTS_SCHEDULE_OWNER   16-bit contractions of 3-D vertex patches: one
 *        launch in which a workgroup owns a tile of 3 x 3 cells (x, y) and a
 *        range of cell layers (z), computes every patch touching its cells
 *        (patches on tile borders are computed by each neighbouring tile) and
 *        sums their corrections in on-chip memory in a fixed order before
 *        updating x once; no staging buffer.  Deterministic.  Other
 *        precisions and cells fall back to FTS_SCHEDULE_STAGED.
 *   FTS_SCHEDULE_AUTO    FTS_SCHEDULE_OWNER on levels of at least 4,096
 *        cells, FTS_SCHEDULE_STAGED below (where one tile launch is too short
 *        to fill the GPU and the staged runs are faster).  The default.
 * Ignored for cells (disjoint, one launch). */
#define FTS_SCHEDULE_STAGED 0
#define FTS_SCHEDULE_COLORED 1
#define FTS_SCHEDULE_OWNER 2
#define FTS_SCHEDULE_AUTO 3
fts_status fts_eigs_set_schedule(fts_eigs *eigs, int32_t schedule);

/* ---- a4: matrix-free SIPG operator --------------------------------------- */

/* y = A x, the SIPG matrix of eq. (bfsipg) on this level (x, y: ndofs FP64,
 * must not alias). */
fts_status fts_apply_operator(const fts_level *level, const double *x, double *y, void *stream);
/* r = b - A x (r must not alias x; may alias b). */
fts_status fts_residual(const fts_level *level, const double *b, const double *x, double *r,
                        void *stream);

/* ---- a5-a9, a12: additive Schwarz smoother --------------------------------- */

/* Workspace bytes fts_schwarz_smooth needs (one residual vector). */
size_t fts_smooth_ws_bytes(const fts_level *level);

/* nsweeps steps of the additive Schwarz smoother, Alg. (addsmoother) with the
 * damping of eq. (additiveschwarz):
 *     r = b - A x;   x <- x + omega * sum_j R_j^T A_j^-1 R_j r
 * with A_j^-1 = (S x..x S) diag(1/Lambda) (S x..x S)^T (eq. fastinverse).
 * Overlapping vertex patches are summed as set by fts_eigs_set_schedule
 * (default FTS_SCHEDULE_AUTO; deterministic).  ws: device workspace of
 * fts_smooth_ws_bytes bytes. */
fts_status fts_schwarz_smooth(const fts_level *level, const fts_eigs *eigs, double omega,
                              fts_prec prec, const double *b, double *x, int32_t nsweeps, void *ws,
                              size_t ws_bytes, void *stream);
/* Only the local-solver part: x <- x + omega * sum_j R_j^T A_j^-1 R_j r. */
fts_status fts_schwarz_apply(const fts_level *level, const fts_eigs *eigs, double omega,
                             fts_prec prec, const double *r, double *x, void *stream);

/* Allocation-free form of fts_schwarz_smooth, for callers that cannot
 * allocate device memory or pass a workspace (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  Same arguments and result
 * as fts_schwarz_smooth without ws / ws_bytes: the residual lives in a static
 * device array of FTS_NOALLOC_SCRATCH_BYTES bytes (32 MiB, i.e. levels of up
 * to 4,194,304 DoFs; each device the library runs on holds its own copy until
 * the process ends), looked up once per device at the first call on it.
 * Larger levels fail with FTS_E_SIZE.  The call allocates nothing.  Every call
 * on one device shares that array: calls that overlap on one device (other
 * streams, other threads) race and must be serialised by the caller; calls
 * ordered on one stream are safe (each call overwrites the whole residual
 * before reading it). */
#define FTS_NOALLOC_SCRATCH_BYTES (32u * 1024u * 1024u)
fts_status fts_schwarz_smooth_noalloc(const fts_level *level, const fts_eigs *eigs, double omega, fts_prec prec,
                                      const double *b, double *x, int32_t nsweeps, void *stream);

/* Multiplicative Schwarz smoother (Alg. multsmoother, eq. coloredschwarz):
 * nsweeps times, for each color c = 0..C-1 in turn: r = b - A x, then
 * x += omega sum_{j in color c} R_j^T A_j^-1 R_j r.  Colors (Sec. 2.3): cells
 * red-black (C = 2); vertex patches the parquet coloring combined with
 * red-black, C = 2^(d+1): color bits t < d are (v_t - 1) mod 2 of the
 * patch's interior vertex v, bit d is sum_t floor((v_t - 1) / 2) mod 2.  Two
 * subdomains of one color share no DoF and their local problems do not
 * couple through A, so each color is one parallel launch updating x in
 * place.  ws: fts_smooth_ws_bytes(level) bytes.  prec as for
 * fts_schwarz_smooth. */
fts_status fts_schwarz_smooth_mult(const fts_level *level, const fts_eigs *eigs, double omega, fts_prec prec,
                                   const double *b, double *x, int32_t nsweeps, void *ws, size_t ws_bytes,
                                   void *stream);

/* ---- a10: transfers and V-cycle ------------------------------------------ */

/* Transfers between a level and its parent (each parent cell = 2^d children,
 * Sec. 2.1).  Prolongation is the embedding of V_{l-1} in V_l: the fine
 * coefficients are the coarse polynomial's values at the fine Gauss-Lobatto
 * nodes; restriction is its transpose (Sec. 2.2).
 * fts_restrict:       bc  = P^T rf   (bc overwritten)
 * fts_prolongate_add: xf += P ec */
fts_status fts_restrict(const fts_level *coarse, const fts_level *fine, const double *rf, double *bc,
                        void *stream);
fts_status fts_prolongate_add(const fts_level *coarse, const fts_level *fine, const double *ec,
                              double *xf, void *stream);

/* Builds nlevels levels by coarsening `finest` (pairs of equal children per
 * axis are merged; every level but the coarsest needs >= 2 cells per axis for
 * vertex patches), 1-D eigen-data of every level > 0, the level vectors, and
 * the FP64 LU factorisation of the coarsest matrix A_0 on the device (no
 * pivoting: A_0 is symmetric positive definite).  The factors are stored by
 * slabs of cells (all cells with one coordinate along the last axis, B
 * unknowns each, nb slabs): A_0 is block tridiagonal over slabs, so L and U
 * are block bidiagonal; the diagonal blocks are kept as the inverses of their
 * triangular factors.  omega_per_level and penalty_per_level: host arrays of
 * nlevels entries, index 0 = coarsest (omega[0] unused); penalty_per_level
 * may be NULL (then the mesh's penalty_factor on every level).  Allocates
 * device memory: 8 (3 nb - 2) B^2 bytes for the coarse factors (plus 8 B^2
 * transiently during setup) and the level vectors. */
fts_status fts_hierarchy_create(const fts_mesh_desc *finest, int32_t nlevels, fts_patch_kind kind,
                                const double *omega_per_level, const double *penalty_per_level,
                                int32_t m_pre, int32_t m_post, fts_hierarchy **out);
fts_status fts_hierarchy_destroy(fts_hierarchy *hier);
/* Level handle l (0 = coarsest), owned by the hierarchy. */
const fts_level *fts_hierarchy_level(const fts_hierarchy *hier, int32_t l);
const fts_eigs *fts_hierarchy_eigs(const fts_hierarchy *hier, int32_t l);

/* x <- MG_L(x, b): one V-cycle of Alg. (gmg) with x as initial guess (pass
 * x = 0 for the preconditioner), prec as in fts_schwarz_smooth.  Returns
 * after the coarse solve on level 0.  b, x: finest-level vectors. */
fts_status fts_vcycle(fts_hierarchy *hier, fts_prec prec, const double *b, double *x, void *stream);

/* ---- a11: outer FP64 CG --------------------------------------------------- */

/* Workspace bytes of fts_pcg: 5 finest-level vectors plus reduction partials. */
size_t fts_pcg_ws_bytes(const fts_hierarchy *hier);

/* Conjugate gradients on the finest level preconditioned by one V-cycle
 * z = MG_L(0, r) (Sec. 2.4), FP64 vectors, residuals and reductions, with the
 * flexible (Polak-Ribiere) beta so that a preconditioner with reduced-
 * precision contractions (prec != FTS_PREC_F64) is tolerated.  x holds the
 * initial guess on entry and the iterate on exit; iterates until
 * ||b - A x|| <= rtol ||b|| or maxit steps.  Dot products are deterministic
 * two-stage reductions; each is read back to the host (the only
 * synchronisations).  history: NULL or maxit+1 doubles of ||r_i||/||b||.
 * iters, relres: NULL or outputs. */
fts_status fts_pcg(fts_hierarchy *hier, fts_prec prec, const double *b, double *x, double rtol,
                   int32_t maxit, void *ws, size_t ws_bytes, int32_t *iters, double *relres,
                   double *history, void *stream);

/* Smoother of the V-cycle on every level > 0: FTS_SMOOTHER_ADDITIVE (default,
 * Alg. addsmoother), FTS_SMOOTHER_MULTIPLICATIVE (Alg. multsmoother with the
 * colors of fts_schwarz_smooth_mult; pre- and post-smoothing run the colors
 * in the same order, as in Sec. 2.4, so the V-cycle is not symmetric: use
 * fts_gmres) or FTS_SMOOTHER_MULTIPLICATIVE_SYMMETRIC (post-smoothing runs
 * the colors in reverse order, the symmetrisation of Sec. 4, so the V-cycle
 * is symmetric and can precondition fts_pcg).  FTS_E_INVAL for other values;
 * fts_vcycle_adjoint needs the additive smoother. */
#define FTS_SMOOTHER_ADDITIVE 0
#define FTS_SMOOTHER_MULTIPLICATIVE 1
#define FTS_SMOOTHER_MULTIPLICATIVE_SYMMETRIC 2
fts_status fts_hierarchy_set_smoother(fts_hierarchy *hier, int32_t smoother);

/* Workspace bytes of fts_gmres: 2 restart + 2 finest-level vectors plus
 * reduction partials. */
size_t fts_gmres_ws_bytes(const fts_hierarchy *hier, int32_t restart);

/* Restarted GMRES on the finest level, right-preconditioned by one V-cycle
 * z = MG_L(0, v) (Sec. 2.4 uses GMRES with the multiplicative smoothers), in
 * the flexible form that keeps the preconditioned directions z_j (so
 * reduced-precision contractions are tolerated): Arnoldi with modified
 * Gram-Schmidt, Givens rotations on the host, x += Z y at the end of each
 * cycle of `restart` steps.  FP64 vectors and deterministic reductions; every
 * inner product is read back (the only synchronisations).  x: initial guess
 * on entry, iterate on exit; stops when the relative residual (least-squares
 * estimate inside a cycle, true residual at its end) is <= rtol or after
 * maxit inner steps.  history: NULL or maxit+1 doubles. */
fts_status fts_gmres(fts_hierarchy *hier, fts_prec prec, const double *b, double *x, double rtol, int32_t restart,
                     int32_t maxit, void *ws, size_t ws_bytes, int32_t *iters, double *relres, double *history,
                     void *stream);

/* Replaces the per-level damping (host array of nlevels, index 0 unused). */
fts_status fts_hierarchy_set_omega(fts_hierarchy *hier, const double *omega_per_level);

/* ---- a14: adjoint of the V-cycle ------------------------------------------- */

/* Allocates the adjoint workspaces of the hierarchy (per level: the inputs of
 * all smoothing steps of one V-cycle, 5 work vectors; small reduction
 * buffers).  Idempotent. */
fts_status fts_hierarchy_enable_adjoint(fts_hierarchy *hier);

/* Reverse mode of one FP64 V-cycle x_out = MG_L(x_in, b) (Alg. gmg).  Recomputes
 * the forward sweeps of the cycle from x_in (instead of storing them across
 * cycles), then propagates lambda_out = dL/dx_out backwards through every
 * smoothing step x' = x + omega_l C_l (b_l - A_l x) (C_l = sum_j R_j^T A_j^-1 R_j),
 * the transfers and the coarse solve.  Outputs:
 *   lambda_b  (device, ndofs; may be NULL)   += dL/db
 *   lambda_x  (device, ndofs; may be NULL)    = dL/dx_in
 *   d_omega   (host, nlevels; may be NULL)   += dL/d omega_l (index 0: 0)
 *   d_penalty (host, nlevels; may be NULL)   += dL/d gamma_hat_l, through the
 *             level operators, the local solvers (d A_j^-1 = -A_j^-1 dA_j A_j^-1,
 *             evaluated in the eigenbasis) and the coarse solve.
 * The matrices are affine in gamma_hat, so dA/dgamma_hat is the penalty part
 * at gamma_hat = 1.  Synchronises the stream once (gradient readback). */
fts_status fts_vcycle_adjoint(fts_hierarchy *hier, const double *b, const double *x_in,
                              const double *lambda_out, double *lambda_b, double *lambda_x,
                              double *d_omega, double *d_penalty, void *stream);

/* x0 = A_0^-1 b0 with the stored LU factorisation, by block forward and
 * backward substitution over the slabs (Alg. gmg, coarse grid solver):
 *   y_0 = inv(L_00) b_0,  y_i = inv(L_ii) (b_i - L_{i,i-1} y_{i-1}),
 *   x_last = inv(U) y_last, x_i = inv(U_ii) (y_i - U_{i,i+1} x_{i+1}),
 * 2 (2 nb - 1) parallel mat-vecs that read 8 B^2 (2 nb - 1) bytes in all
 * (the off-diagonal blocks are half zero and only their nonzero halves are
 * read).  x0 may alias b0.  Solves on one hierarchy must not overlap (they
 * share its workspaces). */
fts_status fts_coarse_solve(fts_hierarchy *hier, const double *b0, double *x0, void *stream);

/* ---- a13: batched smoothing of many meshes of mixed degree ------------------ */

typedef struct fts_batch fts_batch;

/* Builds levels and vertex-patch eigen-data (every patch position has its own
 * 1-D eigenpairs per axis, so anisotropic rectilinear widths are exact) for
 * nmesh independent 3-D meshes of any degrees 1..9, and the work queue of all
 * their patches (meshes in decreasing degree, so the largest local solves are
 * dequeued first).  Vectors of a batch are the meshes' vectors concatenated in
 * mesh order (offsets: fts_batch_mesh_offset).  Allocates the tables, a
 * staging buffer of 2^3 (k+1)^3 doubles per patch and the queue. */
fts_status fts_batch_create(const fts_mesh_desc *meshes, int32_t nmesh, fts_batch **out);
fts_status fts_batch_destroy(fts_batch *batch);
int64_t fts_batch_ndofs(const fts_batch *batch);
fts_status fts_batch_mesh_offset(const fts_batch *batch, int32_t mesh, int64_t *offset, int64_t *ndofs);

/* r = b - A x on every mesh (FP64; one launch per degree present). */
fts_status fts_batch_residual(fts_batch *batch, const double *b, const double *x, double *r,
                              void *stream);
/* x += omega sum_j R_j^T A_j^-1 R_j r on every mesh: ONE persistent launch over
 * the patches of all meshes (workgroups dequeue chunks of one mesh's patches
 * with an atomic counter; a degree switch selects the local solver), then a
 * batched per-cell gather.  prec: FTS_PREC_F64 or FTS_PREC_F32 contractions (update
 * of x in FP64).  Calls on one batch must be stream-ordered (shared staging
 * buffer and counter). */
fts_status fts_batch_apply(fts_batch *batch, double omega, fts_prec prec, const double *r, double *x,
                           void *stream);
/* nsweeps of r = b - A x; x += omega sum_j ...; ws: fts_batch_ws_bytes bytes. */
size_t fts_batch_ws_bytes(const fts_batch *batch);
fts_status fts_batch_smooth(fts_batch *batch, double omega, fts_prec prec, const double *b, double *x,
                            int32_t nsweeps, void *ws, size_t ws_bytes, void *stream);

/* Launch shape of the persistent kernel: threads per workgroup (256 or 512;
 * a thread owns at most two of the N^2 lines of a patch, N = 2(k+1) <= 20),
 * number of persistent workgroups, patches per dequeued chunk (a chunk never
 * spans two meshes). */
fts_status fts_batch_set_launch(fts_batch *batch, int32_t threads, int32_t grid, int32_t chunk);
fts_status fts_batch_get_launch(const fts_batch *batch, int32_t *threads, int32_t *grid,
                                int32_t *chunk);
/* Autotuner: times the persistent kernel (events on `stream`, synchronising)
 * for threads in {256,512} x grid in {1,2,4,8} x (compute units) x chunk
 * in {1,4,16} on the residual r (device, fts_batch_ndofs doubles), keeps the
 * fastest shape and writes a per-candidate report into `report` (may be NULL).
 * Overwrites the batch's staging buffer. */
fts_status fts_batch_autotune(fts_batch *batch, fts_prec prec, const double *r, void *stream,
                              char *report, size_t report_len);

/* ---- Sec. 4: mapped (non-Cartesian) cells, Cartesian surrogate solvers ----- */

/* Logically Cartesian mesh of cells that are the images of the reference cell
 * [0,1]^d under the multilinear map through their 2^d vertices (Sec. 4).
 * vertices: HOST array of prod(ncells[a] + 1) points of dim coordinates each,
 * vertex (v_0, .., v_{d-1}) at index v_0 + (m_0 + 1)(v_1 + (m_1 + 1) v_2), read
 * during the call only.  Cells and DoFs are numbered as on Cartesian meshes. */
typedef struct fts_mapped_desc {
    int32_t dim;            /* 2 or 3 */
    int32_t degree;         /* k: 1..7 in 3-D, 1..15 in 2-D */
    int32_t ncells[3];      /* cells per axis */
    const double *vertices; /* host, prod(ncells + 1) x dim */
    double penalty_factor;  /* gamma_hat > 0 */
} fts_mapped_desc;
typedef struct fts_mapped_level fts_mapped_level;

/* Builds the geometry tables of the mesh (cell volumes |K|, face areas |F|
 * and the penalty of every face, gamma_e = gamma_hat k(k+1)(1/h+ + 1/h-) with
 * h = |K| / |F|, eq. penalty read for mapped cells) and the Cartesian
 * surrogate of every cell (eq. avglength: a box whose width along axis t is
 * the mean length of the cell's edges along t; its faces see the surrogate
 * widths of the neighbours along t): per cell and axis the 1-D SIPG matrices
 * of the box (eq. 1Dsipg) and their generalised eigenpairs (eq.
 * generalizedEVP), uploaded to the current device.  FTS_E_INVAL if a cell map
 * is not orientation preserving. */
fts_status fts_mapped_level_create(const fts_mapped_desc *desc, fts_mapped_level **out);
fts_status fts_mapped_level_destroy(fts_mapped_level *level);
int64_t fts_mapped_level_ndofs(const fts_mapped_level *level);
/* Host copy of the surrogate widths (ncells x dim, cell-major). */
fts_status fts_mapped_surrogate_widths(const fts_mapped_level *level, double *hbar);

/* y = A x with the SIPG form eq. (bfsipg) on the mapped cells: gradients
 * J^-T grad_xi, volume element det J, face normals and area elements from
 * Nanson's formula, (k+1)-point Gauss rule per axis on cells and faces;
 * matrix-free.  r = b - A x for fts_mapped_residual. */
fts_status fts_mapped_apply_operator(const fts_mapped_level *level, const double *x, double *y, void *stream);
fts_status fts_mapped_residual(const fts_mapped_level *level, const double *b, const double *x, double *r,
                               void *stream);

/* Additive cell smoother with the surrogate local solvers (eq. schwarzproj):
 * x += omega sum_K R_K^T Atilde_K^-1 R_K r, Atilde_K^-1 by fast
 * diagonalisation of the surrogate box (eq. fastinverse). */
fts_status fts_mapped_schwarz_apply(const fts_mapped_level *level, double omega, const double *r, double *x,
                                    void *stream);
/* Workspace bytes of fts_mapped_schwarz_smooth (one residual vector). */
size_t fts_mapped_smooth_ws_bytes(const fts_mapped_level *level);
/* nsweeps of r = b - A x; x += omega sum_K R_K^T Atilde_K^-1 R_K r. */
fts_status fts_mapped_schwarz_smooth(const fts_mapped_level *level, double omega, const double *b, double *x,
                                     int32_t nsweeps, void *ws, size_t ws_bytes, void *stream);

/* Multigrid on mapped meshes (Sec. 4 with Alg. gmg).  levels[0..nlevels-1],
 * coarsest first, same dim, degree and penalty factor; level l+1 has twice
 * the cells of level l per axis and its cells are the images of the children
 * of level l's cells under their maps (uniform refinement on the multilinear
 * cell maps, so the spaces are nested and the grid transfers are the
 * reference-cell embeddings of the Cartesian hierarchy).  Smoother on levels
 * l >= 1: omega_per_level[l], m_pre / m_post steps of the additive cell
 * smoother with Cartesian surrogate local solvers; level 0: the mapped
 * operator's own matrix (probed column by column) factored by the slab LU of
 * the Cartesian coarse solver.  Allocates through the registered allocator. */
typedef struct fts_mapped_hierarchy fts_mapped_hierarchy;
fts_status fts_mapped_hierarchy_create(const fts_mapped_desc *levels, int32_t nlevels,
                                       const double *omega_per_level, int32_t m_pre, int32_t m_post,
                                       fts_mapped_hierarchy **out);
fts_status fts_mapped_hierarchy_destroy(fts_mapped_hierarchy *hier);
int64_t fts_mapped_hierarchy_ndofs(const fts_mapped_hierarchy *hier);
/* Smoother on levels >= 1: FTS_SMOOTHER_ADDITIVE (default) or
 * FTS_SMOOTHER_MULTIPLICATIVE, Alg. multsmoother with the surrogate cell
 * solvers and red-black cells (parity of the cell index sum), the residual
 * recomputed before each color; pre-smoothing runs red then black,
 * post-smoothing black then red, so the V-cycle stays symmetric and can
 * precondition fts_mapped_pcg (Sec. 4, Tab. cubedist25mcp).  FTS_E_INVAL for
 * any other value. */
fts_status fts_mapped_hierarchy_set_smoother(fts_mapped_hierarchy *hier, int32_t smoother);
/* Local solvers of the smoother on levels >= 1: FTS_LOCAL_SURROGATE (default,
 * the Cartesian surrogate of eq. avglength by fast diagonalisation) or
 * FTS_LOCAL_EXACT (the inverse of the cell block R_K A R_K^T of the mapped
 * operator, the sACS reference of Tab. cubedist25acp; the blocks are probed
 * from the operator and inverted once, on the first request, and kept:
 * ncells (k+1)^(2d) doubles per level, allocated through the registered
 * allocator).  FTS_E_UNSUPPORTED above 64 unknowns per cell; FTS_E_INVAL for
 * any other value.  Synchronous. */
#define FTS_LOCAL_SURROGATE 0
#define FTS_LOCAL_EXACT 1
fts_status fts_mapped_hierarchy_set_local_solver(fts_mapped_hierarchy *hier, int32_t local);
/* x <- MG_L(x, b) on the finest level. */
fts_status fts_mapped_vcycle(fts_mapped_hierarchy *hier, const double *b, double *x, void *stream);
/* FP64 CG preconditioned by one V-cycle (x = 0 initial guess of the V-cycle),
 * as fts_pcg: stops at ||r|| <= rtol ||b||; history (maxit + 1 doubles, may
 * be NULL) gets ||r_i|| / ||b||; ws: fts_mapped_pcg_ws_bytes bytes. */
size_t fts_mapped_pcg_ws_bytes(const fts_mapped_hierarchy *hier);
fts_status fts_mapped_pcg(fts_mapped_hierarchy *hier, const double *b, double *x, double rtol, int32_t maxit,
                          void *ws, size_t ws_bytes, int32_t *iters, double *relres, double *history,
                          void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FTS_H */
