/*
 * ghsvd.h -- C interface of the MI355X (gfx950) implicit Hari-Zimmermann
 * generalized hyperbolic SVD solver.
 *
 * The method (Singer, Di Napoli, Novakovic, Caklovic, arXiv:1907.08560):
 * given F (m x n), a signature J = diag(+-1) (m entries) and G (p x n) of full
 * column rank, the generalized hyperbolic SVD of Section 3, eq. (3.1), yields
 * the eigenpairs of the Hermitian-definite pencil (H, S) = (F^* J F, G^* G)
 * by eq. (3.2), without forming H or S and without a Cholesky factorization.
 * The solver runs the one-time reduction of Section 5 (hyperbolic QR of F
 * with column pivoting P2, QR of G P2), the one-sided Jacobi-type sweeps of
 * Section 6 (2x2 step of Section 6.1 on a round-robin ordering; optionally
 * the Level-2 blocked variant of Section 6.4 with block transforms applied as
 * matrix-core GEMMs; optionally complex FP32 warm-up sweeps finished in FP64),
 * and the outputs of Section 6.1.7.
 *
 * Conventions for every entry point below:
 *  - Matrices are column-major (LAPACK).  Complex numbers are interleaved
 *    (re, im) doubles; "double *F" of an m x n complex matrix with leading
 *    dimension ldf addresses element (i, j) at F[2 * (i + j * ldf)].
 *  - Matrix, signature and workspace pointers are DEVICE pointers unless a
 *    comment says "host".  The caller owns every buffer; the library keeps no
 *    pointer after a call returns and never modifies inputs.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued on it, and the call returns after the stream has
 *    drained the work it enqueued, so host outputs (info, counters) are valid
 *    on return.
 *  - Return value: 0 success, > 0 warning (outputs valid), < 0 error (device
 *    outputs undefined).  See ghsvd_status.
 *  - The library is thread-safe for calls with distinct workspaces; its only
 *    global state is a mutex-guarded cache of tuned launch parameters
 *    (ghsvd_autotune), the kernel-timing record (ghsvd_profile_enable) and
 *    the scratch array of ghsvd_block_sweeps_noalloc (locked per device).
 */
#ifndef GHSVD_H
#define GHSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GHSVD_OK = 0,
    GHSVD_NOT_CONVERGED = 1, /* sweep cap reached; outputs are the last iterate          */
    GHSVD_EINVAL = -1,       /* bad size, leading dimension, NULL pointer or J entry       */
    GHSVD_ERANK = -2,        /* G numerically rank deficient (or JQR breakdown)           */
    GHSVD_ENONFINITE = -3,   /* NaN or Inf in the inputs or produced during the sweeps    */
    GHSVD_ENOMEM = -4,       /* workspace too small (lwork < ghsvd_workspace_size)       */
    GHSVD_EDEVICE = -5       /* a HIP runtime call failed                                 */
} ghsvd_status;

enum { GHSVD_FP64 = 0, GHSVD_MIXED = 1 };          /* ghsvd_options.precision */
enum { GHSVD_POINTWISE = 0, GHSVD_BLOCKED = 1 };   /* ghsvd_options.variant   */

typedef struct {
    int precision;      /* GHSVD_FP64, or GHSVD_MIXED: complex FP32 warm-up sweeps, then
                           the FP32 transform applied in FP64 and FP64 sweeps finish      */
    int variant;        /* GHSVD_POINTWISE (Section 6.3) or GHSVD_BLOCKED (Section 6.4)   */
    int reduce;         /* 1: reduce to square factors first (Section 5) when m > n or
                           p > n; 0: sweep the tall factors as given                       */
    int block_width;    /* blocked variant: block-column width w (8, 16 or 32); 0 = auto    */
    int waves_per_pair; /* pointwise pair kernel: 64-lane wavefronts per pivot pair
                           (1, 2, 4, 8 or 16); 0 = auto                                    */
    int max_sweeps;     /* sweep cap C_max per precision stage; 0 -> 60 (Algorithm 2 uses
                           ~30 on well-conditioned data; the count grows with cond(S))    */
    int sort;           /* 1: ascending lambda, X's columns permuted alike; 0: unsorted   */
    int crit_literal;   /* 0: criterion (6.12) with sqrt(|h_pp||h_qq|); 1: the printed
                           product form max*eps*sqrt(n)*min                                */
    int inner_order;    /* blocked variant, the inner level per block pivot:
                           GHSVD_INNER_FULL: one sweep over all pairs of the 2w pivot
                           columns in round-robin order (Section 6.4.2, BO);
                           GHSVD_INNER_CROSS (default): the same at the first block step
                           of a sweep, where every block appears once, and only the w x w
                           pairs across the two blocks at the other steps, so each column
                           pair is visited once per sweep; GHSVD_INNER_FB: the Full Block
                           variant (Section 6.4.2), round-robin inner sweeps until one
                           applies no transformation, big or small (Section 6.1.7), at
                           most 30                                                       */
} ghsvd_options;

/* ghsvd_options.inner_order.  GHSVD_INNER_FULL_JQR and GHSVD_INNER_FB_JQR are
 * GHSVD_INNER_FULL and GHSVD_INNER_FB with the block pivots shortened by
 * (J)QR instead of formed as Grams (Section 6.4.2): in the FP64 blocked
 * stage each block pair's c pivot columns F_C, G_C are reduced to square
 * factors F~, G~ (the hyperbolic QR of F_C with the pivoting of Section
 * 5.2.1, its columns put back in pivot-column order, and the QR of G_C), so
 * that F~^* J~ F~ = F_C^* J F_C and G~^* G~ = G_C^* G_C, and the inner level
 * runs the one-sided 2x2 steps of Section 6.1 on them, never squaring the
 * block pivot's conditioning.  A pivot pair that looks numerically dependent
 * is skipped there (left to later block sweeps).  Slower (each block step
 * runs a batched reduction and pointwise sweep of all its block pairs); the
 * FP32 warm-up keeps Gram-formed pivots. */
enum { GHSVD_INNER_FULL = 0, GHSVD_INNER_CROSS = 1, GHSVD_INNER_FB = 2, GHSVD_INNER_FULL_JQR = 3,
       GHSVD_INNER_FB_JQR = 4, GHSVD_INNER_ML_BO = 5, GHSVD_INNER_ML_FB = 6 };
/* GHSVD_INNER_ML_BO and GHSVD_INNER_ML_FB apply the blocking principle once
 * more (Section 6.4 notes it can be applied recursively): each block pair's
 * pivot columns are shortened by (J)QR as for *_JQR, and the shortened
 * pivot (F~, J^, G~) of order 2w is swept by the Level-2 blocked algorithm
 * of block width 8 (block pivots formed as Grams, one full round-robin inner
 * sweep each): one blocked sweep (ML_BO) or blocked sweeps until one applies
 * no big transformation, at most 30 (ML_FB; the nested level re-forms its
 * block pivots every sweep, so it stops like an outer level).  FP64 stage
 * only; the FP32 warm-up uses Gram-formed BO or FB pivots. */

typedef struct {
    int status;
    int sweeps_fp32;           /* FP32 warm-up sweeps (blocked or pointwise)                */
    int sweeps_fp64;           /* FP64 sweeps (blocked plus pointwise)                      */
    int sweeps_blocked;        /* of those, blocked (Level 2) sweeps                        */
    int n2x2;                  /* 2x2 pivots taken by the hyperbolic QR of F                */
    int m_r, p_r;              /* row counts of F and G as swept (n after the reduction)    */
    int n_plus;                /* +1 entries of the signature of the swept F               */
    long long pairs_visited;   /* pivot pairs visited (outer and inner levels)              */
    long long pairs_transformed;
    long long pairs_big;
    long long pw_visited;      /* of the visited pairs, those of the FP64 pointwise sweeps  */
    long long pw_transformed;  /* and of those, the transformed ones                        */
} ghsvd_info;

/* Fills *opt with the defaults: FP64, pointwise, reduce = 1, auto widths,
 * max_sweeps = 60, sort = 1, crit_literal = 0, inner_order = GHSVD_INNER_CROSS. */
void ghsvd_default_options(ghsvd_options *opt);

/* Bytes of device workspace ghsvd_solve needs for an m x n F, p x n G.
 * opt may be NULL (defaults). Returns 0 for invalid sizes. */
size_t ghsvd_workspace_size(int m, int n, int p, const ghsvd_options *opt);

/*
 * Solves (F^* J F) X = (G^* G) X diag(lambda), X^* (G^* G) X = I  (eq. (3.2)).
 *   m, n, p    sizes; require n >= 1, m >= n, p >= n.
 *   F, ldf     device, m x n complex128, ldf >= m.
 *   J          device, m int8 entries, each +1 or -1 (else GHSVD_EINVAL).
 *   G, ldg     device, p x n complex128, ldg >= p, full column rank.
 *   lambda     device, n doubles out: lambda_j = +-(Sigma_F / Sigma_G)^2_j = h_jj / s_jj,
 *              the signed squared generalized hyperbolic singular values.
 *   X, ldx     device, n x n complex128 out, ldx >= n: the S-orthonormal generalized
 *              eigenvectors (column j belongs to lambda_j).
 *   work       device workspace of lwork >= ghsvd_workspace_size(m, n, p, opt) bytes,
 *              256-byte aligned; NULL makes the library allocate and free its own.
 *   opt        host, may be NULL (defaults).
 *   info       host, may be NULL; receives counters and the status.
 * Errors: GHSVD_EINVAL for sizes / ld / NULL / J entries; GHSVD_ERANK when a pivot
 * pair of G is numerically parallel, a column of G vanishes, or the JQR meets a
 * zero J-norm; GHSVD_ENONFINITE for NaN/Inf; GHSVD_ENOMEM for a short workspace.
 */
int ghsvd_solve(int m, int n, int p, const double *F, int ldf, const int8_t *J,
                const double *G, int ldg, double *lambda, double *X, int ldx,
                void *work, size_t lwork, const ghsvd_options *opt, ghsvd_info *info,
                void *stream);

/* Workspace for ghsvd_solve_batched (host arrays m, n, p of length batch). */
size_t ghsvd_workspace_size_batched(int batch, const int *m, const int *n, const int *p,
                                    const ghsvd_options *opt);

/*
 * Many independent pencils (k-points) of uneven order in one call: one
 * reduction per pencil, then all pencils' sweeps run together, each launch
 * covering every still-active pencil; a pencil retires when its own sweep
 * has no big transformation.  m, n, p, ldf, ldg, ldx: host arrays [batch];
 * F, J, G, lambda, X: host arrays [batch] of device pointers (same meaning as
 * ghsvd_solve).  info: host array [batch] (may be NULL).  Returns the worst
 * per-pencil status (an error if any pencil failed, else a warning if any
 * pencil hit the sweep cap, else 0).
 */
int ghsvd_solve_batched(int batch, const int *m, const int *n, const int *p,
                        const double *const *F, const int *ldf, const int8_t *const *J,
                        const double *const *G, const int *ldg, double *const *lambda,
                        double *const *X, const int *ldx, void *work, size_t lwork,
                        const ghsvd_options *opt, ghsvd_info *info, void *stream);

/*
 * Launch tuning for a batch shape (not part of the paper's method: it picks
 * how the same computation is laid onto the GPU).  Runs the one-time
 * reduction and one FP64 pointwise sweep on the given pencils for each
 * wavefronts-per-pair candidate (1, 2, 4, 8), and, for opt->variant ==
 * GHSVD_BLOCKED, one FP64 blocked sweep for each block width (8, 16, 32) with
 * the best wavefront count; the sweep stages are timed with HIP events.  The
 * fastest pair is stored for the shape class (variant, precision, and the
 * base-2 classes of the batch size, the largest n and the largest swept row
 * count); later solves of that class with block_width = 0 or waves_per_pair
 * = 0 use it.  Inputs as ghsvd_solve_batched (device F, J, G; not modified);
 * work/lwork as there (lwork >= ghsvd_workspace_size_batched with
 * block_width = 0; NULL work allocates).  Outputs (host, each may be NULL):
 * *block_width, *waves_per_pair, trial_ms[7] (ms of the pointwise trials
 * for 1, 2, 4, 8 wavefronts, then of the blocked trials for w = 8, 16, 32; -1
 * when not run).  Results of a solve depend on its launch parameters only
 * through rounding.
 */
int ghsvd_autotune(int batch, const int *m, const int *n, const int *p, const double *const *F,
                   const int *ldf, const int8_t *const *J, const double *const *G, const int *ldg,
                   void *work, size_t lwork, const ghsvd_options *opt, int *block_width,
                   int *waves_per_pair, float *trial_ms, void *stream);

/* Drops every tuned launch parameter. */
void ghsvd_autotune_clear(void);

/* ---------------------------------------------------------------------------
 * Component entry points: each runs one stage of the path above, so that a
 * stage can be checked on its own.  Same conventions as ghsvd_solve.
 * ------------------------------------------------------------------------- */

/*
 * One-time reduction (Section 5, eq. (5.1)): hyperbolic QR of F with
 * diagonal plus Bunch-Kaufman partial column pivoting (Section 5.2.1),
 * hyperbolic Householder reflectors (Theorem 5.1, Section 5.3) and the 2x2
 * (J, I) URV pivot step; then the Householder QR of G without pivoting
 * (R_kk = -e^{i arg x_1} ||x||), whose triangular factor R_G is returned
 * with its columns permuted by P2: Gsq = R_G P2.  The iteration sees G
 * only through G^*G, for which this factor and the triangular factor of
 * G P2 (Section 5) are equivalent; the unpivoted QR does not wait for the
 * pivot decisions and runs beside the hyperbolic QR.  Outputs: Fsq (n x n,
 * ldfs >= n, block upper triangular, zeros below), Jsq (n int8), Gsq (n x n,
 * ldgs >= n; Gsq[:, perm^-1] is upper triangular), perm (n ints: column i of
 * F P2 is column perm[i] of F), all device; *n2x2 (host) the number of 2x2
 * pivots.  Then Fsq^* Jsq Fsq = P2^T F^* J F P2 and
 * Gsq^* Gsq = P2^T G^* G P2.
 */
int ghsvd_reduce(int m, int n, int p, const double *F, int ldf, const int8_t *J,
                 const double *G, int ldg, double *Fsq, int ldfs, int8_t *Jsq,
                 double *Gsq, int ldgs, int *perm, int *n2x2, void *stream);

/*
 * The 2x2 step of Section 6.1 for `count` independent pivot pairs (device
 * arrays): a, b, sa, sb real; c, sc complex (interleaved); tol = eps*sqrt(n).
 * Z (device, 8 doubles per pair) receives Z' = D0 Z column-major (z11, z21,
 * z12, z22 as re/im), kind (device int per pair) 0 skipped, 1 small, 2 big,
 * < 0 error (as ghsvd_status).
 */
int ghsvd_pair_params(int count, const double *a, const double *b, const double *c,
                      const double *sa, const double *sb, const double *sc, double tol,
                      int crit_literal, double *Z, int *kind, void *stream);

/*
 * Runs `nsweeps` pointwise FP64 sweeps (or fewer, when a sweep has no big
 * transformation) in place on F (m x n, rows 0..n_plus-1 carry J = +1, the
 * rest J = -1), G (p x n) and Z (n x n, caller-initialized, normally I), on
 * the round-robin ordering of ghsvd_round_robin, waves_per_pair as in
 * ghsvd_options (0 = auto).  counters (host, 3 * nsweeps long longs) gets
 * (visited, transformed, big) per sweep; *sweeps_done (host) the sweeps run.
 */
int ghsvd_sweeps(int m, int n, int p, double *F, int ldf, int n_plus, double *G, int ldg,
                 double *Z, int ldz, int nsweeps, int waves_per_pair, int crit_literal,
                 long long *counters, int *sweeps_done, void *stream);

/*
 * Runs up to `nsweeps` Level-2 blocked FP64 sweeps (Section 6.4, one inner
 * sweep per block pivot) in place on F, G, Z (layout as ghsvd_sweeps) with
 * block width block_width (8, 16 or 32; 0 = auto), stopping after a block sweep
 * without big inner transformations.  Block b holds columns
 * [b w, min(b w + w, n)), nb = ceil(n / w) rounded up to even blocks are
 * paired by ghsvd_round_robin(nb); within a block pair (a, b) the pivot
 * columns are a's then b's, and the inner sweep visits them in
 * ghsvd_round_robin(c) order with tol = eps sqrt(c); inner_order as in
 * ghsvd_options (GHSVD_INNER_CROSS: after the first block step of a sweep,
 * step k pairs column i of block a with column (i + k) mod w of block b).  counters (host,
 * 3 * nsweeps) get (visited, transformed, big) inner pairs per block sweep.
 * Requires n >= 4.
 */
int ghsvd_block_sweeps(int m, int n, int p, double *F, int ldf, int n_plus, double *G, int ldg,
                       double *Z, int ldz, int block_width, int inner_order, int nsweeps,
                       int crit_literal, long long *counters, int *sweeps_done, void *stream);

/*
 * For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid hipMalloc): ghsvd_block_sweeps with the same arguments, results
 * and errors, bit for bit, but without any allocation.  Its scratch
 * (descriptor, done flags, sweep state, counters, partial Grams, block
 * transforms) lives in a library-owned device array of
 * GHSVD_NOALLOC_SCRATCH_BYTES, one copy per GPU, which the library holds
 * until the process ends; the call uses the copy of the current device and
 * looks its address up on the first call there.  F, G, Z are the caller's
 * and swept in place, as in ghsvd_block_sweeps.  The call launches its rounds
 * directly on `stream` (no captured graph, internal stream or timing events)
 * and reads the done flags on the host after every round, so it cannot
 * itself be captured into a graph.
 * Limit: the scratch a call needs grows as (n / w) (m / c + p / c) (2 w)^2
 * complex128 (c = 256 rows, 128 at w = 32) plus O(m + n); a pencil whose need
 * exceeds GHSVD_NOALLOC_SCRATCH_BYTES is rejected with GHSVD_ENOMEM before
 * any work is enqueued (square n = 1024 at every width fits, and n = 2048 at
 * w = 8 and 16).
 * The shortened inner orders (GHSVD_INNER_FULL_JQR, GHSVD_INNER_FB_JQR) are
 * rejected with GHSVD_EINVAL.
 * Calls on one GPU share its array, which keeps the last call's contents (the
 * call clears every counter and state it reads before using it): two calls
 * that overlapped on one GPU would race, so within a process the library
 * holds a per-device lock for the whole call and such calls run one after
 * the other.
 */
#define GHSVD_NOALLOC_SCRATCH_BYTES (32u << 20)
int ghsvd_block_sweeps_noalloc(int m, int n, int p, double *F, int ldf, int n_plus, double *G,
                               int ldg, double *Z, int ldz, int block_width, int inner_order,
                               int nsweeps, int crit_literal, long long *counters,
                               int *sweeps_done, void *stream);

/*
 * Full GHSVD from a finished sweep stage (Phase 4, Section 7, with the
 * outputs of Section 6.1).  Inputs (device, column-major complex128 as
 * interleaved re/im doubles, not modified): the swept F' (m x n, rows
 * 0..n_plus-1 carry J = +1, the rest J = -1), G' (p x n) and the accumulated
 * transformation Z' (n x n) that ghsvd_sweeps or ghsvd_block_sweeps leave in
 * place.  Outputs (device): with h_j = f'_j^* J f'_j, s_j = g'_j^* g'_j and
 * Sigma_j = (|h_j| + s_j)^{1/2},
 *   sigma_f[j] = |h_j|^{1/2} / Sigma_j, sigma_g[j] = s_j^{1/2} / Sigma_j  (n doubles each),
 *   U = F' diag(|h_j|^{-1/2})  (m x n, ldu >= m),
 *   V = G' diag(s_j^{-1/2})    (p x n, ldv >= p),
 *   X = Z^{-1}, Z = Z' diag(Sigma_j)^{-1}  (n x n, ldx >= n),
 * the inverse by LU with complete pivoting (among entries of equal modulus
 * the first in column-major order) and blocked triangular solves.  Then F' Z'^{-1} = U diag(sigma_f) X, G' Z'^{-1} = V diag(sigma_g) X,
 * sigma_f^2 + sigma_g^2 = 1, U^* J U = diag(sign h_j), V^* V = I at
 * convergence, and the eigenvalues of the pencil are sign(h_j) (sigma_f[j] /
 * sigma_g[j])^2.  Errors: GHSVD_EINVAL for sizes, leading dimensions, NULL
 * pointers or n > 4096 (the largest order taken); GHSVD_ERANK when some h_j or s_j is zero or Z is
 * singular (a zero pivot); GHSVD_ENONFINITE for NaN/Inf column norms.
 * work (device, 256-byte aligned, owned by the caller) holds
 * lwork >= ghsvd_full_workspace_size(n) bytes (4 n^2 complex128 + O(n): two
 * working matrices, L and U stored by row and column label, which the solves
 * reuse, plus the inverse diagonal blocks); a shorter lwork gives
 * GHSVD_ENOMEM and a misaligned work GHSVD_EINVAL.  work = NULL makes the
 * call allocate and free its own.  The library keeps no pointer after the
 * call.  Synchronizes the stream (the zero-pivot test is read on the host).
 */
size_t ghsvd_full_workspace_size(int n);  /* 0 for n < 1 or n > 4096 */
int ghsvd_full(int m, int n, int p, const double *F, int ldf, int n_plus, const double *G,
               int ldg, const double *Z, int ldz, double *U, int ldu, double *V, int ldv,
               double *sigma_f, double *sigma_g, double *X, int ldx, void *work, size_t lwork,
               void *stream);

/*
 * The explicit-formation alternative (Section 4.5): H = F^* J F and
 * S = G^* G are formed (FP64 matrix cores) and solved by a Cholesky-based
 * generalized Hermitian eigensolver: S = R^* R, C = R^{-*} H R^{-1},
 * C = V diag(lambda) V^* by blocked two-sided Jacobi (block columns of 16;
 * a 2x2 rotation is applied while |c_pq| exceeds eps sqrt(n) times both
 * sqrt(|c_pp c_qq|) and ||C||_F; the sweeps stop after one without a
 * rotation, at most max_sweeps (0 -> 60)), X = R^{-1} V, lambda ascending.
 * Outputs as ghsvd_solve: H X = S X diag(lambda), X^* S X = I (eq. (3.2)).
 * Forming S squares the conditioning of G, so the eigenvalues carry a
 * relative error of order eps cond(S); the route is taken only when the
 * Cholesky factorization succeeds (every pivot positive and finite) and
 * (max r_ii / min r_ii)^2 <= cond_max, a lower estimate of cond(S).
 * Otherwise, with fallback != NULL, the call runs ghsvd_solve with those
 * options (the implicit HZ path) on the same buffers and returns its status;
 * with fallback == NULL it returns GHSVD_ERANK.
 *   m, n, p, F, ldf, J, G, ldg, lambda, X, ldx as for ghsvd_solve (p >= n;
 *   J entries must be +1 or -1: the fast route reads J > 0 as +1 and does
 *   not check them; the fallback does).
 *   work   device, 256-byte aligned, lwork >= ghsvd_fast_workspace_size(m, n,
 *          p, fallback) (4 n^2 complex128 + O(n^2 / 64), or the fallback's
 *          size if larger); owned by the caller.
 *   info   (host, may be NULL) status, path (GHSVD_PATH_FAST or
 *          GHSVD_PATH_HZ), Jacobi sweeps and rotations, the condition
 *          estimate (0 when the factorization failed) and the fallback's
 *          ghsvd_info.
 * Synchronizes the stream (the factorization's outcome and each sweep's
 * rotation count are read on the host).  Returns GHSVD_OK,
 * GHSVD_NOT_CONVERGED (sweep cap), GHSVD_EINVAL (sizes, NULL pointers,
 * misaligned work), GHSVD_ENOMEM, GHSVD_ERANK (see above) or the fallback's
 * status.
 */
enum { GHSVD_PATH_FAST = 0, GHSVD_PATH_HZ = 1 };
typedef struct {
    int status;
    int path;            /* GHSVD_PATH_FAST or GHSVD_PATH_HZ (the fallback ran) */
    int sweeps;          /* Jacobi sweeps of the fast route                     */
    int pad;
    double cond_est;     /* (max r_ii / min r_ii)^2 of the Cholesky factor      */
    long long rotations; /* 2x2 rotations applied by the fast route             */
    ghsvd_info hz;       /* the fallback's counters when path == GHSVD_PATH_HZ  */
} ghsvd_fast_info;
size_t ghsvd_fast_workspace_size(int m, int n, int p, const ghsvd_options *fallback);
int ghsvd_solve_fast(int m, int n, int p, const double *F, int ldf, const signed char *J,
                     const double *G, int ldg, double *lambda, double *X, int ldx, double cond_max,
                     int max_sweeps, void *work, size_t lwork, const ghsvd_options *fallback,
                     ghsvd_fast_info *info, void *stream);

/*
 * Phase 1 (Section 4): the simultaneous factorizations of the atom blocks.
 *
 * ghsvd_hebpj_batched: ZHEBPJ (Sections 4.2, 4.3) of n_atoms Hermitian
 * matrices T_a of order r (1 <= r <= 512), one workgroup per atom:
 * T_a = Mt_a^* diag(Jt_a) Mt_a by the Hermitian indefinite factorization with
 * Bunch-Parlett complete pivoting (pivot of order 1 when the largest diagonal
 * modulus is at least alpha = (1 + sqrt 17) / 8 times the largest modulus of
 * the Schur complement, else the largest off-diagonal entry as a pivot of
 * order 2; moduli compared squared; ties to the first entry in column-major
 * order), its order-2 pivots diagonalized by a Jacobi rotation and every
 * pivot's rows scaled to signs +-1, the columns put back in the original
 * order (M^ = M P) and the rows permuted stably so that the positive signs
 * come first, then the negative ones.  A Schur complement that is exactly
 * zero ends the factorization: the rest of Mt_a is zero and its signs 0
 * (placed last).
 *   T     device, r x r x n_atoms complex128 (interleaved re/im), T_a
 *         column-major with leading dimension r, atom stride r^2; only the
 *         upper triangle and the real part of the diagonal are read.
 *   Mt    device output, r x r x n_atoms complex128, same layout.
 *   Jt    device output, r x n_atoms int8 (+1, -1, 0).
 *   piv   device output, r x n_atoms int: the index of T_a eliminated at
 *         pivoted position k, stored as -(index + 1) for both positions of an
 *         order-2 pivot.
 *   stats device output, 2 ints per atom: the number of order-2 pivots (or
 *         GHSVD_ENONFINITE when T_a holds a NaN or Inf; Mt_a and Jt_a are
 *         then zero) and the number of zero signs.
 *   work  device, 256-byte aligned, lwork >= ghsvd_hebpj_workspace_size
 *         (2 r^2 n_atoms complex128: the working triangles and the factor rows
 *         in pivot order), owned by the caller.
 * Asynchronous on `stream`; errors returned are only GHSVD_EINVAL (sizes,
 * NULL pointers, misaligned work) and GHSVD_ENOMEM (short workspace).
 *
 * ghsvd_phase1: the per-atom loop of Section 4.4 for n_atoms atoms of
 * 2 nl x n blocks (eq. (4.1), (4.2)): T_a = Mt_a^* Jt_a Mt_a as above,
 * F~_a = Mt_a H_a (FP64 matrix cores), G~_a = [A_a; U_a B_a], stacked by atom.
 *   H     device, m x n complex128, m = 2 nl n_atoms, ldh >= m; rows
 *         2 nl a .. 2 nl a + 2 nl - 1 are H_a = [A_a; B_a].
 *   U     device, nl x n_atoms doubles: column a is the diagonal of U_a.
 *   F, G  device outputs, m x n complex128 (ldf, ldg >= m): F~ and G~.
 *   J     device output, m int8: J~ (per atom: +1 first, then -1, then 0).
 *   stats device output, 2 ints per atom as for ghsvd_hebpj_batched.
 *   work  lwork >= ghsvd_phase1_workspace_size(n_atoms, nl) bytes (the
 *         factorization workspace plus Mt and piv).
 * Then H = F~^* J~ F~ = sum_a H_a^* T_a H_a and S = G~^* G~ = sum_a S_a^* S_a;
 * rows with J~ = 0 are zero rows of F~ and may be dropped before a solve.
 * Asynchronous; errors as above, plus GHSVD_EINVAL for n < 1 or a leading
 * dimension below m.
 */
size_t ghsvd_hebpj_workspace_size(int n_atoms, int r);  /* 0 for bad sizes */
int ghsvd_hebpj_batched(int n_atoms, int r, const double *T, double *Mt, signed char *Jt,
                        int *piv, int *stats, void *work, size_t lwork, void *stream);
size_t ghsvd_phase1_workspace_size(int n_atoms, int nl);  /* 0 for bad sizes */
int ghsvd_phase1(int n_atoms, int nl, int n, const double *T, const double *H, int ldh,
                 const double *U, double *F, int ldf, signed char *J, double *G, int ldg,
                 int *stats, void *work, size_t lwork, void *stream);

/*
 * The round-robin ordering (host): N = n rounded up to even; step s pairs
 * slot N-1 with s and (s+k) mod (N-1) with (s-k) mod (N-1), k = 1..N/2-1;
 * each pair as p < q; a pair meeting index n (odd n) is a bye, p = q = -1.
 * p_out, q_out: host arrays of (N-1) * N/2 ints, step-major.  Returns N-1
 * (the steps per sweep), or -1 for n < 1.
 */
int ghsvd_round_robin(int n, int *p_out, int *q_out);

/*
 * Kernel timing of the sweep kernels, for measurement harnesses.
 * ghsvd_profile_enable(every): from now on every `every`-th launch of each
 * sweep-kernel kind (per process) is bracketed by two HIP events recorded on
 * the stream the kernel is launched on; while it is on, rounds are launched
 * directly instead of through a captured graph.  every <= 0 disables it.
 * ghsvd_profile_read(kind, ...) (host outputs) waits for the recorded events
 * of that kind, returns the summed kernel milliseconds of the timed
 * launches, their count, and the count of all launches of the kind since
 * enabling, then clears that kind's record.  Kinds: GHSVD_PROF_PAIR64 (FP64
 * pointwise pair kernel), GHSVD_PROF_PAIR32 (its FP32 form),
 * GHSVD_PROF_GRAM, GHSVD_PROF_INNER, GHSVD_PROF_UPDATE (the three kernels
 * of an FP64 blocked step), GHSVD_PROF_GRAM32, GHSVD_PROF_INNER32,
 * GHSVD_PROF_UPDATE32 (the same in the FP32 warm-up), GHSVD_PROF_REDUCE (the
 * launches of one column step of the one-time reduction, bracketed
 * together).  Returns GHSVD_EINVAL for an unknown kind.
 */
enum { GHSVD_PROF_PAIR64 = 0, GHSVD_PROF_PAIR32 = 1, GHSVD_PROF_GRAM = 2, GHSVD_PROF_INNER = 3,
       GHSVD_PROF_UPDATE = 4, GHSVD_PROF_GRAM32 = 5, GHSVD_PROF_INNER32 = 6,
       GHSVD_PROF_UPDATE32 = 7, GHSVD_PROF_REDUCE = 8 };
void ghsvd_profile_enable(int every);
int ghsvd_profile_read(int kind, double *ms, long long *timed, long long *launches);

/* Human-readable name of a status value (static storage). */
const char *ghsvd_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* GHSVD_H */
