/*
 * femcg.h -- C ABI of the MI355X (gfx950) Jacobi-PCG library for the
 * P1-P4 finite-element Laplace systems of "Evaluating Accuracy and
 * Efficiency of HPC Solvers for Sparse Linear Systems with Applications to
 * PDEs" (Galizia, Cammarasana, Clematis, Patane).
 *
 * Problem (Sect. 2.2): the Laplace equation with Dirichlet data u = f on the
 * boundary of a 2D/3D domain, discretised on a regular or irregular simplicial
 * mesh, gives a sparse system A u = b whose right-hand side encodes the
 * boundary condition.  Several right-hand sides known a priori form the block
 * system A X = B of Eq. (3) (Sect. 4.3).  Iterations stop when Eq. (2),
 * ||A x - b||_2 / ||b||_2 <= eps, holds; Eq. (1) is the error metric.
 *
 * Conventions shared by every call:
 *  - Plain C types only; no exception crosses the ABI.
 *  - Return value: 0 = ok, > 0 = warning, < 0 = error (FEMCG_E*).  The text of
 *    the last error of the calling thread is fem_last_error().
 *  - "host" pointers are CPU memory owned by the caller; "device" pointers are
 *    HIP device memory (e.g. from a torch CUDA tensor) owned by the caller.
 *    The library never frees caller memory.
 *  - Dense blocks B and X are row-major [n][k] with the k right-hand sides of
 *    a row contiguous ("interleaved"), in the public DOF order below.
 *  - Public DOF order: mesh vertices in mesh order, then (element order
 *    p >= 2) p-1 DOFs per mesh edge, edges in lexicographic order of their
 *    (min, max) vertex pair and the DOF t = 1..p-1 of an edge at
 *    ((p-t) x_min + t x_max) / p (P2: the midpoint, (x_min + x_max) / 2),
 *    then (p = 3, 4) (p-1)(p-2)/2 DOFs per cell, cells in mesh order; inside
 *    a cell with vertices (v0, v1, v2) the lattice points
 *    (a0 x_v0 + a1 x_v1 + a2 x_v2) / p, a0 + a1 + a2 = p, all a > 0, in
 *    decreasing lexicographic order of (a0, a1, a2).  Solver vectors hold the
 *    free (non-Dirichlet) DOFs in increasing DOF index.
 *    Internal row permutations of the sparse formats are never visible.
 *  - A fem_matrix owns its workspaces: calls that use the same matrix must
 *    not overlap (from several threads, or on several streams at once).
 *    Different matrices are independent.  The serve_* calls of one server
 *    must come from one thread at a time (its assembly worker runs beside
 *    them on its own).
 *  - "stream" is a hipStream_t (NULL = the null stream).  Device work is
 *    enqueued on it; calls that must inspect device state synchronise it.
 */
#ifndef FEMCG_H
#define FEMCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FEMCG_OK 0
#define FEMCG_WARN_MAXITER 1     /* some column hit max_iter; stats hold its residual */
#define FEMCG_EINVAL (-1)        /* invalid argument */
#define FEMCG_EMESH (-2)         /* invalid mesh: non-positive element measure, bad index */
#define FEMCG_ENOMEM (-3)        /* host or device allocation failed */
#define FEMCG_EBREAKDOWN (-4)    /* p.Ap <= 0 or a non-finite scalar in some column */
#define FEMCG_EUNSUPPORTED (-5)  /* unsupported order, dimension, k or format */
#define FEMCG_EDEVICE (-6)       /* a HIP runtime call failed */
#define FEMCG_EADMIT (-7)        /* serving: request does not fit the memory budget */

#define FEMCG_MAX_K 64           /* right-hand sides per solve */

/* Sparse formats of the solver copy of A. */
#define FEM_FORMAT_CSR 0
#define FEM_FORMAT_SELL 1        /* SELL-C-sigma, rows sorted by length in windows of sigma */
#define FEM_FORMAT_AUTO 2        /* chosen by the autotuner (fem_tune) */
#define FEM_ORDER_SFC 0x10       /* flag for fem_set_format: internal rows in Morton
                                    (Z-curve) order of the DOF coordinates */
#define FEM_ASSEMBLE_DEVICE 0x100 /* flag for fem_assemble: assemble on the device */
#define FEM_ASSEMBLE_HOST_ONLY 0x200 /* flag for fem_assemble: host system and solver copy
                                        only, no device memory (fem_dofs / fem_csr / fem_free
                                        work without a GPU; calls that need the device
                                        return FEMCG_EINVAL) */

/* Arithmetic of the Krylov iteration. */
#define PCG_FP64 0               /* FP64 values, vectors and dots */
#define PCG_MIXED 1              /* FP32 inner PCG (FP64 dots) inside FP64 iterative refinement */

/* A simplicial mesh (Sect. 2.2 input domain).  All arrays are host memory,
 * read during fem_assemble only. */
typedef struct {
    int32_t dim;                  /* 2 (triangles) or 3 (tetrahedra) */
    int64_t nverts;
    const double *coords;         /* [nverts][dim] */
    int64_t ncells;
    const int32_t *cells;         /* [ncells][dim+1], positively oriented */
    const uint8_t *on_boundary;   /* [nverts], 1 = Dirichlet vertex */
} fem_mesh;

/* Opaque assembled system; owns its host and device buffers. */
typedef struct fem_matrix fem_matrix;

typedef struct {
    double tol;            /* Eq. (2) threshold eps (per column) */
    int64_t max_iter;      /* cap on products A p per column; 0 = 20 sqrt(n) log2(n) + 100 */
    int32_t precision;     /* PCG_FP64 or PCG_MIXED */
    double inner_eta;      /* PCG_MIXED: relative residual reduction of each inner solve */
    int32_t check_every;   /* iterations per device graph replay between host polls */
    int32_t use_x0;        /* 1: X holds the initial guess; 0: start from zero */
    int32_t max_restarts;  /* restarts after the true residual misses tol (drift) */
    int32_t max_outer;     /* PCG_MIXED: cap on refinement steps */
    int32_t use_graph;     /* 1: replay the iterations as a HIP graph */
} pcg_opts;

typedef struct {
    int64_t n;             /* free DOFs (rows of A) */
    int64_t nnz;           /* structural nonzeros of A */
    int64_t nnz_nonzero;   /* entries kept by the solver copy (numerically nonzero) */
    int64_t nnz_stored;    /* entries stored, padding included */
    int32_t k;             /* right-hand sides of the last solve */
    int32_t status;        /* return code of the last solve */
    int32_t precision;
    int32_t format;
    int32_t outer;         /* refinement steps (PCG_MIXED) or restarts + 1 (PCG_FP64) */
    int32_t graph_replays;
    int64_t iters[FEMCG_MAX_K];     /* products A p per column (inner ones for PCG_MIXED) */
    double relres[FEMCG_MAX_K];     /* true FP64 residual of Eq. (2) per column */
    double setup_s;        /* fem_assemble wall time */
    double solve_s;        /* pcg_solve wall time, entry to converged result */
    double bytes;          /* algorithmic HBM bytes of the iterations */
    double gbps;           /* bytes / solve_s / 1e9 */
    double gflops;         /* algorithmic flops / solve_s / 1e9 */
    double footprint_mb;   /* device memory held by the matrix and its workspaces */
} pcg_stats_t;

/* Fill opts with defaults: tol 1e-8, precision FP64, inner_eta 1e-4,
 * check_every 32, use_x0 0, max_restarts 3, max_outer 30, use_graph 1. */
void pcg_default_opts(pcg_opts *opts);

/* Assemble the stiffness matrix K_ij = integral grad(phi_i).grad(phi_j) of
 * the P1 (order 1) or P2 (order 2) Lagrange basis on triangles or tetrahedra,
 * or of the P3 / P4 basis on triangles (Table 7's degrees 3 and 4; order 3 or
 * 4 on a tetrahedral mesh is FEMCG_EUNSUPPORTED) -- the sign-
 * flipped, symmetric counterpart of the paper's Laplacian matrix (Sect. 2.2:
 * cotangent weights w(i,j), diagonal -sum w) -- and eliminate the Dirichlet
 * DOFs (zero source): A = K_II, b = -K_ID g_D.  Builds the solver copy
 * (entries with |a| <= 4 eps64 max_row|a| dropped, FP64 and FP32 values,
 * inverse diagonal) in `format` and uploads it to the current device.
 * Mesh arrays are copied; *out is owned by the caller until fem_free.
 * With FEM_ASSEMBLE_DEVICE in `format`, the DOF numbering, the Dirichlet
 * marking, the element matrices and the summation of the element entries
 * (in the same element order) run on the current device, on the null
 * stream, with temporary device memory of about 32 bytes per element entry
 * (cells * nloc^2); meshes beyond its index ranges (3D P2 with 2^21 or more
 * vertices, 2^31 or more element entries) are assembled on the host.
 * With FEM_ASSEMBLE_HOST_ONLY (excludes FEM_ASSEMBLE_DEVICE) nothing is
 * uploaded and no HIP call is made: fem_dofs, fem_csr, pcg_stats and fem_free
 * work without a GPU, and every call that needs the device copy returns
 * FEMCG_EINVAL.
 * Errors: FEMCG_EINVAL, FEMCG_EMESH (non-positive element), FEMCG_ENOMEM,
 * FEMCG_EUNSUPPORTED, FEMCG_EDEVICE. */
int fem_assemble(const fem_mesh *mesh, int32_t order, int32_t format, fem_matrix **out);

/* Statistics of one bicgstab_solve. */
typedef struct {
    int64_t iters;         /* BiCGStab iterations (two products with A each; one
                              for the last if it stops at the half step) */
    double relres;         /* true FP64 ||b - A x|| / ||b|| (Eq. (2)) */
    int32_t restarts;      /* restarts from x: the true residual missed tol, or a
                              Lanczos near-breakdown |(rh, r)| <= 1e-14 ||rh|| ||r|| */
    int32_t block_size;
    int64_t nblocks;
    double setup_s;        /* block inverses and upload (first call per block size) */
    double solve_s;        /* wall time of the call */
    double bytes;          /* algorithmic HBM bytes of the iterations */
} bicgstab_stats_t;

/* The paper's iterative solver (Sect. 3.2: BiCGStab with a Block-Jacobi
 * preconditioner) on A = K_II: BiCGStab, right preconditioned by Block-Jacobi
 * with exact blocks of block_size (1..64) consecutive free DOFs in the public
 * order (the last block may be shorter; block_size 1 is Jacobi).  One
 * right-hand side, FP64, zero initial guess.  Stops when the recursive
 * residual satisfies Eq. (2) (||r|| <= tol ||b||), also at the half step
 * (||s|| <= tol ||b||), then checks the true residual and restarts from x
 * when it misses tol (at most 3 times).  A Lanczos near-breakdown,
 * |(rh, r)| <= 1e-14 ||rh|| ||r||, restarts it from x with rh = r (at most
 * 100 times).
 * row_scale: NULL, or host [n_free] FP64 in the public order, every entry
 * finite and > 0 (copied): the solver then runs on the row-scaled system
 * D A x = D b with D = diag(row_scale), whose solution is the same.  With
 * D = B^-1, B the lumped mass (for P1 the area or volume of the cells
 * around each vertex), this is the paper's nonsymmetric A = B^-1 L
 * (Sect. 2.2).  The blocks, the residuals, the Eq. (2) test and the
 * reported relres are those of the scaled system; all ones gives the
 * unscaled solve bit for bit.
 * B, X: device [n_free] FP64, public order (B read, X written).  max_iter:
 * cap on iterations, 0 = 20 sqrt(n) log2(n) + 100.  The block inverses
 * (Gauss-Jordan with partial pivoting, on the host) are built at the first
 * call with a given block size and row scale and kept with A until the
 * format, the block size or the row scale changes.  Work is enqueued on `stream` and the call synchronises it.
 * stats may be NULL.
 * Returns 0 (the true residual meets Eq. (2)), FEMCG_WARN_MAXITER (it does
 * not: the iteration cap was reached, or the third restart still missed tol;
 * stats hold the residual), or FEMCG_EINVAL (arguments), FEMCG_EBREAKDOWN
 * (a singular block, rho = 0, (rh, v) = 0, omega = 0 or a non-finite
 * scalar), FEMCG_ENOMEM, FEMCG_EDEVICE. */
int bicgstab_solve(fem_matrix *A, const double *B, double *X, double tol, int32_t block_size,
                   const double *row_scale, int64_t max_iter, void *stream, bicgstab_stats_t *stats);

/* ---- direct solver: sparse Cholesky of A = K_II (Sect. 4.3) ----
 * Sect. 4.3 sets an iterative solver's time for t right-hand sides,
 * T_IS_PC + t T_IS_SOLVE, against a direct solver's T_FACT + t T_SOLVE: the
 * matrix is factorised once and each right-hand side costs a forward and a
 * backward triangular solve (one at a time or as the block of Eq. (3)).
 * A is symmetric positive definite, so the factorisation is Cholesky,
 * A(perm, perm) = L L^T, by the multifrontal method on a nested-dissection
 * order computed from the DOF coordinates (Sect. 3.1: the direct solvers
 * reorder the matrix to limit the fill-in before factorising it). */
typedef struct fem_chol fem_chol;   /* opaque: ordering, tree and factor (device) */

typedef struct {
    int64_t n;             /* rows of A */
    int64_t nnz_l;         /* entries of L (lower triangle, diagonal included) */
    int32_t nodes;         /* nested-dissection tree nodes (fronts) */
    int32_t levels;        /* tree depth + 1 */
    int32_t max_front;     /* largest frontal matrix (rows) */
    int32_t pad;
    double flops;          /* factorisation flops (POTRF + TRSM + SYRK of every front) */
    double factor_mb;      /* device memory of the factor panels */
    double work_mb;        /* peak device memory of two consecutive levels of fronts */
    double order_s;        /* host: nested-dissection ordering */
    double symbolic_s;     /* host: update sets, tree levels (after chol_factor also the
                              factor's host set-up and its uploads) */
    double factor_s;       /* numeric factorisation on the device (0 until chol_factor) */
    double total_s;        /* chol_factor wall time: ordering, symbolic, set-up, numeric */
    double solve_s;        /* last chol_solve, call to result */
} chol_stats_t;

/* Ordering and symbolic analysis only, on the host (works on a host-only
 * matrix): fills out; perm_out (may be NULL) receives n_free entries, the
 * free row at each position of the elimination order.  Returns 0,
 * FEMCG_EINVAL (NULL), FEMCG_ENOMEM. */
int chol_analyze(const fem_matrix *A, chol_stats_t *out, int32_t *perm_out);

/* Factorise A = K_II (device copy needed): ordering and symbolic analysis on
 * the host, numeric factorisation on stream (synchronised on return).  Every
 * front keeps its diagonal block inverted (L11^-1, also stored transposed),
 * so that chol_solve applies them as matrix products; the factor is
 * otherwise the Cholesky factor L of A(perm, perm).  *out
 * receives a library-owned factor, independent of A afterwards; free it with
 * chol_free.  Returns 0, FEMCG_EINVAL (NULL, host-only matrix),
 * FEMCG_EBREAKDOWN (a non-positive pivot: A not positive definite),
 * FEMCG_ENOMEM, FEMCG_EDEVICE. */
int chol_factor(fem_matrix *A, fem_chol **out, void *stream);

/* X = A^-1 B for k right-hand sides as one block (Eq. (3)): B, X device
 * [n_free][k] FP64 in the public order (X may not alias B); forward and
 * backward substitution with the factor on stream (synchronised on return).
 * Allocates its work vectors per call.  Returns 0, FEMCG_EINVAL,
 * FEMCG_ENOMEM, FEMCG_EDEVICE. */
int chol_solve(fem_chol *L, const double *B, double *X, int32_t k, void *stream);

/* Statistics of the factor and of its last solve.  Returns 0 or FEMCG_EINVAL. */
int chol_stats(const fem_chol *L, chol_stats_t *out);

void chol_free(fem_chol *L);

/* Sizes and DOF data of the discretisation (Sect. 2.2: P1 DOFs are the mesh
 * vertices; Table 7's degrees add p-1 DOFs per edge and (p-1)(p-2)/2 per
 * cell), in the public DOF order above.  Any output pointer may be NULL.
 * n_all: every DOF; n_free: the non-Dirichlet DOFs, the solver's unknowns.
 * dof_coords: host [n_all][dim]; dirichlet: host [n_all] (1 = the DOF lies
 * on the boundary, where u = f is imposed); free2dof: host [n_free] (the DOF
 * index of each solver row).  Works on a host-only matrix.  Returns 0 or
 * FEMCG_EINVAL (A NULL). */
int fem_dofs(const fem_matrix *A, int64_t *n_all, int64_t *n_free, double *dof_coords,
             uint8_t *dirichlet, int64_t *free2dof);

/* Host copy of the assembled A = K_II (structural pattern, unpruned, FP64)
 * in CSR with columns ascending: rowptr [n_free+1], col [nnz], val [nnz].
 * Pass NULL arrays to query nnz only. */
int fem_csr(const fem_matrix *A, int64_t *nnz, int64_t *rowptr, int32_t *col, double *val);

/* B = -K_ID g_D (Sect. 2.2: b encodes the boundary condition).
 * g_all: host [n_all][k], Dirichlet data at every DOF (only Dirichlet DOFs
 * are read).  B: device [n_free][k], FP64.  Enqueued on stream. */
int fem_rhs(const fem_matrix *A, const double *g_all, int32_t k, double *B, void *stream);

/* Y = A X for k interleaved columns (Sect. 3.2's MatMult, here as SpMM).
 * X, Y: device [n_free][k] FP64, public order.  Enqueued on stream. */
int fem_spmv(fem_matrix *A, const double *X, double *Y, int32_t k, void *stream);

/* fem_spmv without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, layout and result as fem_spmv (the same
 * kernels and tiling: Y is identical bit for bit).  Every buffer beyond X and
 * Y (launch table, state, per-tile partials, the permuted copies of X and Y)
 * lives in one fixed device array of FEMCG_NOALLOC_SCRATCH_BYTES per device,
 * which each device that runs it holds until the process ends.  Fully
 * asynchronous on stream: the call enqueues four kernels and returns, with no
 * host copy and no synchronisation.  All calls on one device share that
 * array, so calls that overlap on one device (other streams, other threads)
 * race: serialise them, e.g. on one stream.  A must have a device copy.
 * Returns 0, FEMCG_EINVAL (NULL argument, host-only matrix, or a product
 * needing more scratch than the limit: about n_free * pad(k) <= 4M, pad(k)
 * = k rounded up to a power of two), FEMCG_EUNSUPPORTED (k outside
 * 1..FEMCG_MAX_K), FEMCG_EDEVICE. */
#define FEMCG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int fem_spmv_noalloc(fem_matrix *A, const double *X, double *Y, int32_t k, void *stream);

/* Solve A X = B column by column with Jacobi-preconditioned CG (Sect. 2.1's
 * preconditioned system with M = diag(A)), stopping each column when Eq. (2)
 * holds for its recursive residual and then confirming it with the true FP64
 * residual (restart from X when it drifted).  B, X: device [n_free][k] FP64
 * (X: initial guess when opts->use_x0, else overwritten).  opts NULL =
 * defaults with opts.tol = tol.  Blocks the host until the solve has
 * converged or stopped; X is ready when stream reaches the end of the call.
 * Returns 0, FEMCG_WARN_MAXITER, or an error (FEMCG_EBREAKDOWN, ...). */
int pcg_solve(fem_matrix *A, const double *B, double *X, int32_t k, double tol,
              const pcg_opts *opts, void *stream);

/* Many independent systems in one batch: every CG phase of every system runs
 * in one persistent kernel launch (systems are independent; results do not
 * depend on which other systems share the batch).  Arrays of length nsys;
 * all systems use opts->precision.  Status per system in status[]. */
int pcg_solve_batch(int32_t nsys, fem_matrix *const *A, const double *const *B, double *const *X,
                    const int32_t *k, const double *tol, const pcg_opts *opts, int32_t *status,
                    void *stream);

/* Statistics of the last solve on this matrix (Sect. 2.3's measures:
 * execution time, FLOPS and memory, beside the iterations and the accuracy
 * of Eq. (2) per column as relres, the true FP64 ||b - A x|| / ||b||;
 * Eq. (1) needs a ground-truth solution and is left to the caller).  The fields are described with
 * pcg_stats_t.  Works on a host-only matrix (sizes only).  Returns 0 or
 * FEMCG_EINVAL (A or out NULL). */
int pcg_stats(const fem_matrix *A, pcg_stats_t *out);

/* Autotune the solver copy for k right-hand sides: times SpMM over candidate
 * formats (CSR; SELL with C in {16,32,64}, sigma in {1, 64, 1024}) on the
 * device and keeps the fastest (3D and P2 meshes also try the Morton row order).
 * Returns the chosen format, FEM_ORDER_SFC included; C_out and sigma_out
 * may be NULL. */
int fem_tune(fem_matrix *A, int32_t k, int32_t precision, int32_t *C_out, int32_t *sigma_out,
             void *stream);

/* What pcg_tune chose, and the times it compared. */
typedef struct {
    int32_t format, C, sigma, sfc; /* solver copy: FEM_FORMAT_CSR/SELL, slice height, sigma, Morton order */
    int32_t lpr;                   /* SpMM lanes per row at one column (1, 2, 4 or 8) */
    int32_t band;                  /* tiling mode: 0 tiles, 1 band, 2 single-workgroup loop */
    int32_t tile;                  /* fem_set_tiling's tile argument chosen (0 for band 2) */
    int32_t ntiles;                /* tiles per vector in that mode */
    int32_t precision;             /* PCG_FP64 or PCG_MIXED: the faster to tol */
    int32_t fp64_fallback;         /* 1: no mixed solve beat FP64 (or none reached tol) */
    double inner_eta;              /* fastest mixed inner tolerance (0: none reached tol) */
    double fp64_ms, mixed_ms;      /* time to tol: FP64, and the fastest mixed solve */
} pcg_tune_report;

/* Autotune the whole solve of k right-hand sides B (device [n_free][k],
 * public order) to tol (Eq. (2)), for later solves of the same kind:
 *  1. the solver-copy format and row order, as fem_tune (SpMM time);
 *  2. at k = 1, the SpMM lanes per row (1, 2, 4, 8; SpMM time);
 *  3. the tile size of the phase kernels in the automatic tiling mode: the
 *     default, half and double (time of 128 capped FP64 iterations);
 *  4. the precision and the mixed inner tolerance: one FP64 solve and
 *     mixed solves with inner_eta in {1e-2, 1e-3, 1e-4, 1e-5}, each to tol,
 *     timed from call to result.
 * The matrix keeps the chosen format, tiling and lanes per row; opts (in:
 * the caller's options; out: precision and inner_eta set to the fastest
 * solve, FP64 when no mixed solve is faster) and report are filled.  Runs
 * solves on stream and synchronises; allocates a temporary X.  Returns 0,
 * FEMCG_EINVAL (arguments, or the FP64 solve misses tol), or the errors of
 * fem_tune and pcg_solve. */
int pcg_tune(fem_matrix *A, const double *B, int32_t k, double tol, pcg_opts *opts, pcg_tune_report *report,
             void *stream);

/* Rebuild the solver copy in an explicit format (SELL: slice height C in
 * {8,16,32,64}, sorting window sigma >= 1).  format may carry FEM_ORDER_SFC:
 * the internal row order then follows a Morton curve through the DOF
 * coordinates before the sigma sort, so rows processed together share
 * gathered neighbours (3D grids); the public DOF order is unchanged. */
int fem_set_format(fem_matrix *A, int32_t format, int32_t C, int32_t sigma);

/* Tiling of the iteration kernels.  band = 0: large tiles, every block of a
 * phase reduces all tile partials of the previous phase at its start (small
 * systems); band = 1: small tiles swept by each XCD's blocks as one band of
 * rows, partial sums folded by the blocks that complete each group of tiles
 * (large systems); band = 2: the whole iteration loop of the system in one
 * 1024-thread workgroup (p in LDS, no launch per phase; needs n * kp <= 4096,
 * kp = k rounded up to a power of two, else pcg_solve fails with
 * FEMCG_EINVAL); band = -1: automatic (band 2 when it fits, else band 1 for
 * vectors above 64 MB, else band 0).  tile: rows per tile target count
 * (band 0) or bytes of one FP64 vector slice per tile (band 1); 0 = default
 * (band 1: 16..64 KB, sized for about 4096 tiles).
 * Drops cached workspaces. */
int fem_set_tiling(fem_matrix *A, int32_t band, int32_t tile);

/* Time one hot kernel of the iteration on the workspace of the last solve
 * (same launch configuration as inside the solve): `reps` full iterations
 * (SpMM, update, p-update, every column forced active) run on `stream`, so
 * the caches hold what they hold inside a solve; each launch of the chosen
 * kernel records its start and end into HIP events from its dispatch packet
 * (hipExtLaunchKernel), the times a kernel trace reports.  kernel: 0 = SpMM + p.q, 1 = fused
 * update, 2 = p-update.  Writes the mean duration in ms and the algorithmic
 * bytes of one launch.  Overwrites the workspace vectors (not B or X). */
int pcg_time_kernel(fem_matrix *A, int32_t kernel, int32_t reps, void *stream, double *ms,
                    double *bytes);

/* Cold-cache SpMM rate (the MatMult of Sect. 3.2 as an SpMM, timed so that
 * no copy is cache-resident): builds the SpMM launch of each of the nmat matrices for
 * k right-hand sides in `precision` on its own workspace (p zero-filled),
 * launches all once, then times `reps` rounds of launching them in turn,
 * so with copies totalling far more than the 256 MB last-level cache every
 * launch starts cold.  Host pointers; the matrices stay owned by the caller.
 * *ms = mean duration of one launch, *bytes = mean algorithmic bytes of one
 * launch (numerically nonzero entries, values + int32 column indices + row
 * pointers or slice lengths, p read once and q written once).  Overwrites the
 * workspace vectors of the matrices (not B or X of any caller). */
int pcg_time_spmm_cold(int32_t nmat, fem_matrix *const *A, int32_t k, int32_t precision, int32_t reps,
                       void *stream, double *ms, double *bytes);

void fem_free(fem_matrix *A);

/* Thread-local text of the last error ("" if none). */
const char *fem_last_error(void);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of solve requests (Sect. 4.3's multiple
 * independent systems, arriving over time).  A server owns a device memory
 * budget; requests are admitted while their footprint fits, run as slots of
 * the persistent batched kernels, and retire when converged, freeing their
 * memory for waiting requests.
 * ------------------------------------------------------------------------- */
typedef struct fem_server fem_server;

typedef struct {
    int64_t id;
    int32_t status;         /* solve status */
    int32_t k;
    int64_t n;
    int64_t iters_max;      /* max over columns */
    double t_submit;        /* seconds on the server clock */
    double t_ready;         /* host assembly finished */
    double t_admit;         /* admitted to the device */
    double t_done;
    double relres_max;
    double footprint_mb;    /* device memory the request held against the budget
                               (0 if it never had a footprint: failed assembly) */
} fem_request_info;

/* budget_bytes: device memory the server may hold for admitted requests.
 * max_slots: systems resident at once.  precision: PCG_FP64 or PCG_MIXED. */
int serve_create(double budget_bytes, int32_t max_slots, int32_t precision, int32_t check_every,
                 fem_server **out);

/* Submit a request: the server assembles it (host), queues it and admits it
 * when memory frees up.  g_all: host [n_all][k].  Returns the request id
 * (>= 0) or an error.  The server takes ownership of nothing the caller
 * passes (arrays are copied). */
int64_t serve_submit(fem_server *s, const fem_mesh *mesh, int32_t order, const double *g_all,
                     int32_t k, double tol);

/* Advance the server by one tick: admit what fits, run check_every
 * iterations of every resident system as one batched graph replay, retire
 * converged systems.  Returns the number of requests still queued or running. */
int serve_step(fem_server *s);

/* 1 if request id is done; then X (host [n_free][k], may be NULL) and info
 * are filled and the request's memory is released. */
int serve_poll(fem_server *s, int64_t id, double *X, fem_request_info *info);

/* Server clock (seconds since serve_create). */
double serve_clock(const fem_server *s);

void serve_destroy(fem_server *s);

#ifdef __cplusplus
}
#endif

#endif /* FEMCG_H */
