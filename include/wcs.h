/*
 * wcs — sparse Cholesky for compressed wavelet Galerkin matrices on MI355X.
 *
 * C ABI of the library.  The operations follow the problem statement of
 * Harbrecht & Multerer, "A fast direct solver for nonlocal operators in
 * wavelet coordinates":
 *   - Section 4: a nested dissection ordering P of the symmetric sparsity
 *     pattern (computed once per pattern and reusable for every matrix with
 *     that pattern, as done for V_J and A_J in Section 6.1), then the
 *     Cholesky factorization P A P^T = L L^T;
 *   - Section 1 and Section 5: the factor used as an exact inverse of the
 *     compressed matrix, factored once and applied to many right-hand sides
 *     (Section 5.1) and many time steps (Section 5.2);
 *   - Section 5.3: the half solve with L^T alone, used to draw Gaussian
 *     random field samples (here in precision form, x = P^T L^-T z, whose
 *     covariance is A^-1).
 *
 * Conventions shared by all calls
 *   Pattern: lower triangle including the diagonal, compressed sparse column,
 *     colptr int64[n+1] (colptr[0] = 0), rowind int32[colptr[n]], rows strictly
 *     ascending within a column and the diagonal stored first.  Host memory,
 *     owned by the caller, copied by wcs_analyze.
 *   Values: device FP64 array aligned with rowind (one value per stored
 *     entry), owned by the caller.
 *   Right-hand sides / solutions: device FP64, column-major n x nrhs with
 *     leading dimension ld >= n, always in the caller's (original) ordering;
 *     the permutation is internal.
 *   Workspace: device memory provided by the caller (the library performs no
 *     device allocation); its size comes from wcs_workspace_size.
 *   Streams: every device call is enqueued on the given HIP stream and is
 *     asynchronous unless stated otherwise.
 *   Errors: status codes (wcs_status); no C++ exception crosses the ABI.
 *     wcs_last_error() returns a thread-local human-readable detail.
 *   Handles are owned by the caller and released only by the *_free calls.
 */
#ifndef WCS_H
#define WCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *wcs_stream; /* a hipStream_t; NULL = the default stream */

typedef struct wcs_symbolic_s *wcs_symbolic; /* host: ordering, trees, supernodes, plan */
typedef struct wcs_factor_s *wcs_factor;     /* device-resident L plus its plan */

typedef enum {
    WCS_OK = 0,
    WCS_EINVAL = -1,    /* malformed argument or pattern */
    WCS_ENOMEM = -2,    /* workspace too small, or host allocation failed */
    WCS_EHIP = -3,      /* a HIP runtime call failed */
    WCS_ENOTSPD = -4,   /* a pivot was not positive (or NaN): matrix not SPD */
    WCS_ENOTCONV = -5,  /* iterative refinement did not reach the tolerance */
    WCS_ESTATE = -6,    /* call not valid in the handle's current state */
    WCS_ESINGULAR = -7  /* a zero (or non-finite) pivot in an LU factorization */
} wcs_status;

typedef enum {
    WCS_FP64 = 0,       /* fronts stored and factored in FP64 */
    WCS_FP32 = 1,       /* fronts stored and factored in FP32 (FP64 diagonal
                           tiles in fronts with at least fp64_diag_min_cols pivots) */
    WCS_LU64 = 2        /* nonsymmetric matrix with the analysed (symmetric) pattern:
                           P A P^T = L U without pivoting, L unit lower and U upper
                           triangular, both in FP64 fronts (wcs_factor_numeric_lu) */
} wcs_precision;

typedef enum {
    WCS_SOLVE_FULL = 0, /* X = A^-1 B          = P^T L^-T L^-1 P B */
    WCS_SOLVE_L = 1,    /* X = L^-1 P B         (result in pivot order) */
    WCS_SOLVE_LT = 2    /* X = P^T L^-T B       (input in pivot order)  */
} wcs_part;

/* Products with the factor itself, P A P^T = L L^T (see wcs_apply). */
typedef enum {
    WCS_APPLY_L = 1,    /* X = P^T L B          (input in pivot order)  */
    WCS_APPLY_LT = 2    /* X = L^T P B          (result in pivot order) */
} wcs_apply_part;

typedef struct {
    int32_t leaf_size;          /* nested dissection stops at <= leaf_size vertices (default 64) */
    double dense_degree_frac;   /* peel vertices whose degree >= dense_degree_frac * n ... */
    double dense_degree_min;    /* ... and >= dense_degree_min; peeled vertices join the root separator
                                   (defaults 0.25 and 1024) */
    const double *coords;       /* optional n x coord_dim row-major vertex positions used only to
                                   choose the split of each dissection step; the separator itself
                                   is always a vertex cover of the cut edges of the graph.
                                   NULL = graph-only (breadth-first level structure) splits */
    int32_t coord_dim;          /* 1..3 when coords != NULL */
    const int32_t *user_perm;   /* optional ordering (perm[k] = original index of pivot k);
                                   bypasses nested dissection */
    int32_t relax;              /* 1 = relaxed supernode amalgamation (default), 0 = fundamental only */
} wcs_analyze_opts;

typedef struct {
    int32_t n;
    int64_t nnz_lower;          /* stored entries of the input (lower triangle incl. diagonal) */
    int64_t nnz_l;              /* nnz(L), lower triangle including the diagonal, from the
                                   fundamental symbolic structure */
    int64_t flops;              /* sum over columns of colcount^2 (fundamental structure) */
    int64_t flops_padded;       /* the same sum over the amalgamated supernodes actually factored */
    int32_t nsuper_fund;        /* fundamental supernodes */
    int32_t nsuper;             /* supernodes after amalgamation (= fronts) */
    int32_t nlevels;            /* levels of the assembly tree (height + 1) */
    int32_t max_front;          /* largest front order m */
    int32_t nsep_nodes;         /* nodes of the separator tree */
    int32_t npeeled;            /* dense vertices moved into the root separator */
    int64_t front_elems;        /* sum over fronts of ld*m, ld = m rounded up to 8 (front storage, elements) */
    int64_t nnz_l_padded;       /* entries of L as stored by the fronts (explicit zeros included) */
    int32_t nseg;               /* independent diagonal blocks: 1, or the instances of a batch */
} wcs_symbolic_info_t;

typedef struct {
    int32_t iterations;         /* refinement steps taken */
    double raw_residual;        /* max column relative residual after the first low-precision solve */
    double final_residual;      /* max column ||b - A x||_2 / ||b||_2 at exit */
} wcs_ir_report;

/* Status name ("WCS_OK", ...). */
const char *wcs_status_string(int status);
/* Detail of the last failing call on this thread (empty string if none). */
const char *wcs_last_error(void);

/*
 * Ordering and symbolic analysis (host only, synchronous, deterministic).
 * Validates the pattern (WCS_EINVAL on any violation of the conventions
 * above), builds the adjacency graph (Section 4), orders it by nested
 * dissection (or takes opts->user_perm), and computes the elimination tree,
 * column counts (Lemma 4.1 pattern), fundamental and amalgamated supernodes,
 * the assembly tree, extend-add index maps and the level schedule.
 * opts may be NULL (defaults).  On success *out owns a new handle.
 */
int wcs_analyze(int32_t n, const int64_t *colptr, const int32_t *rowind,
                const wcs_analyze_opts *opts, wcs_symbolic *out);

int wcs_symbolic_info(wcs_symbolic sym, wcs_symbolic_info_t *info);

/*
 * Copies the symbolic results into caller host arrays (each may be NULL):
 *   perm[n]              perm[k] = original index of pivot k
 *   parent[n]            elimination tree, parent[j] = min{i > j : l_ij != 0} or -1
 *   colcount[n]          nonzeros of column j of L (diagonal included)
 *   super_ptr[nsuper_fund+1]  first column of each fundamental supernode
 *   sep_tree[6*nsep_nodes]    nested dissection tree, node t = (lo, mid, sep, hi,
 *                        child1, child2) in pivot positions: V1 = perm[lo:mid],
 *                        V2 = perm[mid:sep], S = perm[sep:hi]; leaves have mid = -1
 */
int wcs_symbolic_export(wcs_symbolic sym, int32_t *perm, int32_t *parent, int32_t *colcount,
                        int32_t *super_ptr, int32_t *sep_tree);

/*
 * Relaxed (factored) supernode partition: relaxed_ptr[nsuper+1] first columns,
 * and front_order[nsuper] = m (rows of each front).  Either may be NULL.
 */
int wcs_symbolic_fronts(wcs_symbolic sym, int32_t *relaxed_ptr, int32_t *front_order);

/*
 * Batch of independent systems (many uneven instances at once).  Combines the
 * analyses parts[0..count-1] (each from wcs_analyze, unchanged and still owned
 * by the caller) into one handle for the block-diagonal matrix
 * diag(A_0, ..., A_{count-1}): instance b occupies the unknowns
 * [seg_ptr[b], seg_ptr[b+1]) in both the original and the pivot order, its
 * stored entries follow those of instance b-1 (values of the batch = the
 * instances' value arrays concatenated in order, rows shifted by seg_ptr[b]),
 * and right-hand sides stack the instances' rows.  The assembly forest is the
 * union of the instances' trees, so a factorization, solve or refinement of
 * the batch handle runs the fronts of equal tree height of every instance in
 * the same launches: the leaf fronts of all instances together first, then
 * each level above across all instances.  Each instance's factor is exactly
 * the one its own handle would give.  Refinement tests the tolerance per
 * instance and column (wcs_factor_residuals).  Host only; *out owns a new
 * handle independent of the parts.
 */
int wcs_symbolic_batch(int32_t count, const wcs_symbolic *parts, wcs_symbolic *out);
/* seg_ptr[nseg+1]: first unknown of every instance (nseg from wcs_symbolic_info; 1 for a single matrix). */
int wcs_symbolic_segments(wcs_symbolic sym, int32_t *seg_ptr);

void wcs_symbolic_free(wcs_symbolic sym);

/*
 * Device workspace (bytes) needed by wcs_factor for this pattern, precision
 * and number of right-hand sides solved at once (max_nrhs >= 1).  The same
 * workspace serves the factor, its solves and the refinement.
 */
int wcs_workspace_size(wcs_symbolic sym, wcs_precision prec, int32_t max_nrhs, size_t *bytes);

/*
 * Numeric factorization P A P^T = L L^T (Section 4) of the matrix with the
 * analysed pattern and the device FP64 values values_dev.  The factor lives in
 * the workspace (caller-owned device memory of at least the size from
 * wcs_workspace_size, 256-byte aligned), which must stay valid until
 * wcs_factor_free.  values_dev is read during this call's device work only.
 * If bad_col is non-NULL the call waits for the stream and reports the first
 * failing pivot (pivot order, -1 if none) and returns WCS_ENOTSPD when one
 * failed; with bad_col NULL the call is asynchronous and wcs_factor_check
 * reports the outcome later.
 */
int wcs_factor_create(wcs_symbolic sym, wcs_precision prec, int32_t max_nrhs,
                      void *workspace, size_t bytes, wcs_stream stream, wcs_factor *out);
int wcs_factor_numeric(wcs_factor f, const double *values_dev, wcs_stream stream, int32_t *bad_col);

/*
 * LU factorization (Section 5.1: the PCM system matrix of eq:PCM2 is not
 * symmetric; Section 6.1 factors it by LU on the nested dissection ordering
 * of its symmetric pattern) of a factor created with WCS_LU64:
 * P A P^T = L U without pivoting, L unit lower triangular, U upper
 * triangular; the pattern of L is that of the Cholesky factor and U's the
 * transposed one.  lower_dev: device FP64 values of A on and below the
 * diagonal, aligned with the analysed lower pattern (A[r][c] for the stored
 * entry (r, c), r >= c); upper_dev: the values above the diagonal in the same
 * positions (A[c][r] for the stored (r, c); the diagonal positions are not
 * read).  No pivoting: the matrix must admit the factorization (for example
 * by strict diagonal dominance by columns); a zero or non-finite pivot gives
 * WCS_ESINGULAR with its pivot position in *bad_col (when bad_col is non-NULL,
 * as for wcs_factor_numeric; otherwise wcs_factor_check reports it).
 * wcs_solve on an LU factor: WCS_SOLVE_FULL gives X = A^-1 B =
 * P^T U^-1 L^-1 P B, WCS_SOLVE_L gives L^-1 P B (pivot order), WCS_SOLVE_LT
 * gives P^T U^-1 B (input in pivot order).  wcs_factor_export returns the
 * columns of L (unit diagonal stored); wcs_factor_export_upper the same
 * columns of U^T (entry (i, j) of the export is u(j, i)), in the same
 * format.  The products, refinement, SpMV, theta-scheme, gradient, profile
 * and autotune calls are for Cholesky factors and return WCS_EINVAL on an
 * LU factor.  Asynchronous on the stream unless bad_col is non-NULL.
 */
int wcs_factor_numeric_lu(wcs_factor f, const double *lower_dev, const double *upper_dev, wcs_stream stream,
                          int32_t *bad_col);
int wcs_factor_export_upper(wcs_factor f, int32_t j0, int32_t j1, int64_t *Up, int32_t *Ui, double *Ux,
                            wcs_stream stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc and provide
 * no workspace): wcs_factor_create without a workspace argument.  The factor
 * lives in a static device array of WCS_STATIC_WORKSPACE_BYTES that the
 * library holds on every GPU it runs on until the process ends; the call
 * allocates no device memory and creates no stream or event (every later
 * call on this factor runs all its launches on the stream it is given, with
 * no look-ahead or auxiliary stream).  The static array belongs to the
 * current device and serves one factor at a time: WCS_ESTATE while another
 * factor created by this call on the same device is alive (wcs_factor_free
 * releases it), WCS_ENOMEM (with the needed size in wcs_last_error) when
 * wcs_workspace_size for sym, prec and max_nrhs exceeds
 * WCS_STATIC_WORKSPACE_BYTES.  The array keeps the last factor's contents;
 * every numeric factorization clears what it needs.  Calls on such a factor
 * that overlap in time on one GPU (different streams or threads) race.
 * All other calls take the factor as they take one from wcs_factor_create and
 * give the same results.  Synchronous (plan tables are copied on `stream`).
 */
#define WCS_STATIC_WORKSPACE_BYTES (64u << 20)
int wcs_factor_create_static(wcs_symbolic sym, wcs_precision prec, int32_t max_nrhs, wcs_stream stream,
                             wcs_factor *out);
/* Waits for the stream; *bad_col = first failing pivot or -1; returns WCS_ENOTSPD if one failed. */
int wcs_factor_check(wcs_factor f, wcs_stream stream, int32_t *bad_col);
void wcs_factor_free(wcs_factor f);
/*
 * Relative residuals ||b - A x||_2 / ||b||_2 of the last wcs_solve_refined on
 * this factor, per instance and column: rel[b * nrhs + c] for instance b of
 * nseg (nseg = 1 for a single matrix).  count = capacity of rel (>= nseg*nrhs).
 * WCS_ESTATE if no refinement has run.  Host memory; synchronous.
 */
int wcs_factor_residuals(wcs_factor f, double *rel, int64_t count);

/*
 * Replay mode.  With enable != 0, wcs_factor_numeric records its whole launch
 * sequence into a HIP graph the first time it runs with a given values_dev
 * pointer and replays that graph afterwards (a different pointer records
 * again); the triangular sweeps of wcs_solve and wcs_solve_refined are
 * recorded once per (part, nrhs) the same way.  The recorded sequences hold
 * kernel launches only.  Recording needs a created stream: calls on the NULL
 * stream run their launches directly.  enable = 0 drops the recorded graphs.
 * Host only (the recorded graph is replayed on the call's stream).
 */
int wcs_factor_use_graphs(wcs_factor f, int enable);

/* Trailing-update kernels (per level of the assembly tree). */
typedef enum {
    WCS_UPD_REG128 = 0,     /* 128 x 128 tiles, operands staged through registers into LDS */
    WCS_UPD_REG64 = 1,      /* 64 x 64 tiles (one wave per tile), same staging */
    WCS_UPD_STREAM128 = 2,  /* 128 x 128 tiles, operands streamed global -> LDS, four chunks in flight */
    WCS_UPD_STREAM128_3 = 3,/* the same with three chunks in flight: less LDS, one more workgroup per CU */
    WCS_UPD_STREAM128_K32 = 4 /* 128 x 128 tiles streamed in two chunks of 32 (FP32) / 16 (FP64) k-columns:
                                 half the barriers per product */
} wcs_update_variant;

/*
 * Autotuner for the trailing-update kernel.  Factors values_dev (which leaves
 * a valid factor, as wcs_factor_numeric does) ten times on the stream: a
 * warm-up and a timed run with each wcs_update_variant on every level, timing
 * each level of the assembly tree with HIP events; then keeps, per level, the
 * fastest variant.  All variants compute bitwise the same factor (same
 * products in the same order).  Synchronous.  tiles (nlevels entries, may be
 * NULL) receives the choice per level; ms (2 entries, may be NULL) the summed
 * level times with the default variant (WCS_UPD_STREAM128 for FP64 fronts,
 * WCS_UPD_REG128 for FP32) and with the chosen ones.  Drops a recorded
 * factorization graph.
 */
int wcs_factor_autotune(wcs_factor f, const double *values_dev, wcs_stream stream, int32_t *tiles, double *ms);
/* Sets the update kernel per level (nlevels wcs_update_variant values), e.g. from an earlier autotune. */
int wcs_factor_set_tiles(wcs_factor f, const int32_t *tiles);

/*
 * Diagnostic: performs one numeric factorization (as wcs_factor_numeric with
 * bad_col NULL) with a HIP event pair around every kernel launch on `stream`,
 * waits for it, and fills stats[WCS_NKCLASS], one entry per kernel class:
 *   0 front zero-fill, 1 value scatter, 2 extend-add, 3 panel (diagonal block
 *   factor + triangular solve), 4 panel with FP64 diagonal blocks (FP32
 *   factors), 5 trailing update on the matrix cores.
 * Each entry holds the launch count, the summed event time and the
 * algorithmic work of those launches (flops: multiply-add = 2; bytes: data the
 * operation must move once).  The events add a little time between launches.
 */
#define WCS_NKCLASS 6
typedef struct {
    int32_t launches;
    double ms;
    double flops;
    double bytes;
} wcs_kernel_stat;
int wcs_factor_profile(wcs_factor f, const double *values_dev, wcs_stream stream, wcs_kernel_stat *stats);

/*
 * Diagnostic: as wcs_factor_profile, but timing whole levels of the schedule
 * (level 0 = leaves, nlevels-1 = root; a front's level is its height in the
 * assembly tree, or for fronts with at least WCS_LATE_MIN_PIVOTS pivots
 * (environment, default 1024) one below its parent's level) with one event
 * pair around all launches of a level (extend-add and dense steps).
 * levels[h] gets the level's time and the algorithmic flops of its fronts
 * (sum over pivots of the squared column length of the factored front).
 * nlevels entries.
 */
int wcs_factor_profile_levels(wcs_factor f, const double *values_dev, wcs_stream stream, wcs_kernel_stat *levels);

/*
 * Copies columns [j0, j1) (pivot order) of L to host memory in compressed
 * sparse column form over the stored (amalgamated) pattern, explicit zeros
 * included: Lp[j1-j0+1] offsets starting at 0, Li row indices (pivot order,
 * ascending, diagonal first), Lx values as FP64.  The caller sizes Li/Lx from
 * a first call with Li = Lx = NULL, which fills Lp only.  Synchronous.
 */
int wcs_factor_export(wcs_factor f, int32_t j0, int32_t j1, int64_t *Lp, int32_t *Li, double *Lx,
                      wcs_stream stream);

/*
 * Triangular solves with the factor (Section 5: factor once, solve many).
 * B_dev: device FP64, n x nrhs column-major, ld >= n, overwritten in place by
 * the result (see wcs_part).  1 <= nrhs <= max_nrhs of the factor.
 * In FP32 factors the solve runs in FP32 on an FP32 copy of B (one rounding
 * of B to FP32 and of the result back to FP64).
 */
int wcs_solve(wcs_factor f, wcs_part part, int32_t nrhs, double *B_dev, int64_t ld, wcs_stream stream);

/*
 * Products with the factor (Section 5.3: the Gaussian field is drawn by
 * multiplying white noise with the Cholesky factor of the covariance matrix;
 * here x = P^T L z has covariance P^T L L^T P = A).  WCS_APPLY_L: X = P^T L B
 * with B in pivot order; WCS_APPLY_LT: X = L^T P B with the result in pivot
 * order; so APPLY_L(APPLY_LT(B)) = A B and APPLY_L(SOLVE_L(B)) = B up to
 * rounding.  B_dev: device FP64, n x nrhs column-major, ld >= n, overwritten
 * in place; 1 <= nrhs <= max_nrhs.  FP32 factors compute in FP32 (one rounding
 * of B to FP32 and of the result back).  Asynchronous on the stream; uses the
 * factor's right-hand-side buffers, so calls on one factor are ordered by the
 * stream like its solves.  Errors: WCS_EINVAL for bad arguments,
 * WCS_ESTATE before a numeric factorization.
 */
int wcs_apply(wcs_factor f, wcs_apply_part part, int32_t nrhs, double *B_dev, int64_t ld, wcs_stream stream);

/*
 * X = A^-1 B by iterative refinement against the FP64 input matrix:
 * X0 = solve(B); repeat R = B - A X (FP64), stop when every column has
 * ||R||_2 / ||B||_2 <= tol, else X += solve(R) — at most max_iter corrections.
 * Each correction solves with R scaled per column by a power of two (R stays
 * inside the FP32 range, unscaling is exact).  FP32 factors with nrhs = 8,
 * 16, 32 or 64 form R from the FP32 solve outputs instead of X: R = B - A X0,
 * then R -= A D after each correction D (FP64 products and sums); this equals
 * B - A X up to the FP64 rounding of the sums X + D (about eps |A| |X|), so
 * tol should stay well above eps times the condition number.  When that
 * updated residual meets tol by less than a factor 100, R is formed once more
 * from X itself (FP64) and that residual decides; rep->final_residual and
 * wcs_factor_residuals report the residual the decision used.  values_dev are
 * the FP64 values used by the factorization (same pattern).  Reads the
 * residual norms back to the host once per step (synchronous).  Returns
 * WCS_ENOTCONV (with *rep filled, and X_dev holding the last iterate) if tol
 * is not reached.
 */
int wcs_solve_refined(wcs_factor f, const double *values_dev, int32_t nrhs, const double *B_dev,
                      double *X_dev, int64_t ld, double tol, int32_t max_iter, wcs_ir_report *rep,
                      wcs_stream stream);

/*
 * Y = A X for the FP64 input matrix (full symmetric A from its stored lower
 * triangle), device arrays, n x nrhs column-major with leading dimension ld.
 */
int wcs_spmv(wcs_factor f, const double *values_dev, int32_t nrhs, const double *X_dev, double *Y_dev,
             int64_t ld, wcs_stream stream);

/*
 * Theta scheme in time (Section 5, eq:theta): G (u_{i+1} - u_i) / dt - L ((1 - theta) u_i
 * + theta u_{i+1}) = (1 - theta) f_i + theta f_{i+1}, taken in an L2-orthonormal
 * wavelet basis (mass matrix G = I) with L = -K for a symmetric positive definite
 * operator matrix K.  The matrix of every step is A = I + theta dt K; theta = 1/2
 * is Crank-Nicolson.
 *
 * wcs_theta_matrix: A_values_dev[e] = theta dt K_values_dev[e], plus 1 on the
 * diagonal entries, for the stored lower pattern of the factor's analysis
 * (device FP64 arrays of nnz_lower entries; A_values_dev may be K_values_dev).
 * Factor A with wcs_factor_numeric before the steps.  Errors: WCS_EINVAL for
 * theta outside (0, 1], dt <= 0 or null pointers.  Asynchronous on the stream.
 *
 * wcs_theta_steps: nsteps steps over the factor of A; A_values_dev are the values
 * it was factored from.  F_dev: f at the nsteps + 1 times, n x (nsteps + 1)
 * column-major with leading dimension ldf >= n.  U_dev: n x (nsteps + 1)
 * column-major with leading dimension ldu >= n; column 0 holds u_0 on entry,
 * columns 1..nsteps receive u_1..u_nsteps.  Each step forms the explicit part
 * from A as (u_i - (1 - theta) A u_i) / theta (one SpMV) and solves once with
 * the factor (FP64), or refines that solve to tol against A (FP32 factors, at most
 * ten corrections per step; *rep gets the largest iteration count, raw and
 * final residual over the steps; FP64 factors report 0 and -1).  Synchronous
 * per refinement step for FP32 factors, else asynchronous.  Errors: WCS_EINVAL
 * (bad arguments), WCS_ESTATE (no numeric factorization), WCS_ENOTCONV (a step
 * missed tol; U holds the steps before it).
 */
int wcs_theta_matrix(wcs_factor f, const double *K_values_dev, double theta, double dt, double *A_values_dev,
                     wcs_stream stream);
int wcs_theta_steps(wcs_factor f, const double *A_values_dev, double theta, double dt, int32_t nsteps,
                    const double *F_dev, int64_t ldf, double *U_dev, int64_t ldu, double tol, wcs_ir_report *rep,
                    wcs_stream stream);

/*
 * Gaussian random field samples in covariance form (Section 5.3,
 * eq:CholFastField): out = G^-1 (abar^G + L X), the wavelet coefficients of
 * the field a_J = Psi_J G^-1 (abar^G + L X), where L L^T = C^G is the
 * Cholesky decomposition of the Galerkin covariance matrix and G the mass
 * matrix.  cov: a Cholesky factor of C^G (its own ordering P_C, so L =
 * P_C^T L_C); mass: a Cholesky factor of G created from its own analysis
 * (Section 6.3: the mass matrix gets an ordering of its own, with much less
 * fill than the system matrix's), on the same index set (equal n).  Either
 * may be FP64 or FP32 (FP32 products and solves round once to FP32 and back).
 * X_dev: nrhs standard normal vectors, n x nrhs column-major with leading
 * dimension ldx, read as coefficients in cov's pivot order (white noise: any
 * fixed order gives the same distribution).  abar_dev: the mean term in the
 * original order, n x nrhs with leading dimension lda, or one vector for all
 * samples (lda = 0), or NULL (no mean).  out_dev: n x nrhs, leading dimension
 * ld, original order; it may be X_dev when ldx == ld.  nrhs may not exceed
 * either factor's max_nrhs.  Uses both factors' right-hand-side buffers, so
 * calls on them are ordered by the stream.  Errors: WCS_EINVAL (bad arguments,
 * LU factors, different n), WCS_ESTATE (a factor without numeric values).
 * Asynchronous on the stream.
 */
int wcs_field_sample(wcs_factor cov, wcs_factor mass, int32_t nrhs, const double *abar_dev, int64_t lda,
                     const double *X_dev, int64_t ldx, double *out_dev, int64_t ld, wcs_stream stream);

/*
 * Gradient of a scalar loss through x = A^-1 b with respect to the stored
 * lower entries of A, given lam = A^-1 (dloss/dx): entry (i,j), i > j, gets
 * -(lam_i x_j + lam_j x_i); a diagonal entry gets -lam_i x_i.  Device arrays:
 * lam_dev[n], x_dev[n], gA_dev[nnz_lower] (aligned with the pattern).
 */
int wcs_grad_pattern(wcs_factor f, const double *lam_dev, const double *x_dev, double *gA_dev,
                     wcs_stream stream);


#ifdef __cplusplus
}
#endif
#endif /* WCS_H */
