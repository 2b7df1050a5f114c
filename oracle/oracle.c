/*
 * CPU oracle for the sparse Cholesky path — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded FP64 code that defines what the GPU library
 * must compute.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it; the library itself never does.  It shares no code,
 * header or table with the library.
 *
 * What is computed (Harbrecht & Multerer, "A fast direct solver for nonlocal
 * operators in wavelet coordinates"):
 *   - Section 4: for a symmetric permutation P (pi), the Cholesky factor of
 *     P A P^T = L L^T, lower triangular with positive diagonal (unique).
 *   - Lemma 4.1: without cancellation, l_ij != 0 (i > j) iff a path from i to
 *     j exists whose interior vertices are all numbered below min(pi(i),pi(j)).
 *     The symbolic part below computes exactly that pattern through the
 *     elimination tree (parent[j] = min{i > j : l_ij != 0}) and row subtrees
 *     (row i of L = union of the tree paths from each k with C_ik != 0, k < i,
 *     up to i).
 *   - Section 1 / Section 5: the factor is used as an exact inverse:
 *     x = P^T L^-T L^-1 P b, and the half solves L^-1 P b and P^T L^-T z
 *     (the latter draws a Gaussian field with covariance A^-1, cf. Section 5.3),
 *     and the products with the factor itself, P^T L b and L^T P b: the
 *     sampling of Section 5.3 multiplies white noise by the Cholesky factor
 *     of the covariance matrix, so that x = P^T L z has covariance A.
 *   - Section 4 nested dissection: V = V1 u V2 u S with no edge between V1
 *     and V2, ordered V1, V2, S, recursively; orc_check_nd verifies that
 *     block structure for a given ordering and separator tree.
 *
 * Conventions: A is given by its lower triangle in compressed sparse column
 * form (colptr int64[n+1], rowind int32[nnz], rows ascending, diagonal
 * present).  perm[k] is the original index of the k-th pivot, so
 * C = P A P^T has C[k][l] = A[perm[k]][perm[l]].  Dense right-hand sides are
 * column-major n x nrhs with leading dimension ld.
 *
 *   - Section 5.1 (eq:PCM2) and Section 6.1: the nonsymmetric system
 *     matrix of the polarizable continuum model is factored by LU on the
 *     same ordering; its pattern is symmetric, so L has the Cholesky pattern
 *     and U the transposed one.  orc_lu computes P A P^T = L U without
 *     pivoting (L unit lower triangular, U upper triangular), orc_lu_solve
 *     x = P^T U^-1 L^-1 P b, orc_gemv the product with the nonsymmetric A.
 *
 * Return codes: 0 ok, -1 invalid input, -2 out of memory, -4 not positive
 * definite (first bad pivot column in *bad_col, pivot order), -5 a zero (or
 * non-finite) pivot in the LU factorization (column in *bad_col).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ENOTSPD -4
#define ORC_ESINGULAR -5

/* inverse permutation; returns -1 if perm is not a bijection of 0..n-1 */
static int invert_perm(int32_t n, const int32_t *perm, int32_t *iperm)
{
    for (int32_t i = 0; i < n; i++) iperm[i] = -1;
    for (int32_t k = 0; k < n; k++) {
        int32_t o = perm[k];
        if (o < 0 || o >= n || iperm[o] != -1) return -1;
        iperm[o] = k;
    }
    return 0;
}

int orc_check_perm(int32_t n, const int32_t *perm)
{
    int32_t *ip = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!ip) return ORC_ENOMEM;
    int r = invert_perm(n, perm, ip);
    free(ip);
    return r == 0 ? ORC_OK : ORC_EINVAL;
}

/*
 * Strictly-lower row lists of C = P A P^T: for each row i (pivot order), the
 * columns k < i with C[i][k] != 0.  rp has n+1 entries, ri holds the lists.
 */
static int build_row_lists(int32_t n, const int64_t *colptr, const int32_t *rowind,
                           const int32_t *iperm, int64_t **rp_out, int32_t **ri_out)
{
    int64_t *rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!rp) return ORC_ENOMEM;
    for (int32_t j = 0; j < n; j++) {
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int32_t i = rowind[p];
            if (i == j) continue;
            int32_t a = iperm[i], b = iperm[j];
            int32_t hi = a > b ? a : b;
            rp[hi + 1]++;
        }
    }
    for (int32_t i = 0; i < n; i++) rp[i + 1] += rp[i];
    int32_t *ri = (int32_t *)malloc(sizeof(int32_t) * (size_t)(rp[n] > 0 ? rp[n] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!ri || !fill) { free(rp); free(ri); free(fill); return ORC_ENOMEM; }
    memcpy(fill, rp, sizeof(int64_t) * ((size_t)n + 1));
    for (int32_t j = 0; j < n; j++) {
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int32_t i = rowind[p];
            if (i == j) continue;
            int32_t a = iperm[i], b = iperm[j];
            int32_t hi = a > b ? a : b, lo = a > b ? b : a;
            ri[fill[hi]++] = lo;
        }
    }
    free(fill);
    *rp_out = rp;
    *ri_out = ri;
    return ORC_OK;
}

/*
 * Elimination tree and column counts of L for C = P A P^T.
 *   parent[j]   = min{ i > j : l_ij != 0 } or -1
 *   colcount[j] = number of nonzeros of column j of L, diagonal included
 *   *nnzL       = sum colcount,  *flops = sum colcount^2
 * The row pattern of row i is the union of the tree paths from each k in
 * row i of C (k < i) up to i; walking each path until a node already seen for
 * this row visits every (i, j) with l_ij != 0 exactly once.
 */
int orc_symbolic(int32_t n, const int64_t *colptr, const int32_t *rowind, const int32_t *perm,
                 int32_t *parent, int32_t *colcount, int64_t *nnzL, int64_t *flops)
{
    if (n < 0) return ORC_EINVAL;
    int32_t *iperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *anc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!iperm || !anc || !mark) { free(iperm); free(anc); free(mark); return ORC_ENOMEM; }
    if (invert_perm(n, perm, iperm)) { free(iperm); free(anc); free(mark); return ORC_EINVAL; }
    int64_t *rp = NULL;
    int32_t *ri = NULL;
    int rc = build_row_lists(n, colptr, rowind, iperm, &rp, &ri);
    if (rc) { free(iperm); free(anc); free(mark); return rc; }

    /* elimination tree with path compression through 'anc' */
    for (int32_t i = 0; i < n; i++) {
        parent[i] = -1;
        anc[i] = -1;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            int32_t r = ri[p];
            while (anc[r] != -1 && anc[r] != i) {
                int32_t next = anc[r];
                anc[r] = i;
                r = next;
            }
            if (anc[r] == -1) {
                anc[r] = i;
                parent[r] = i;
            }
        }
    }
    /* row subtrees -> column counts */
    for (int32_t i = 0; i < n; i++) { colcount[i] = 0; mark[i] = -1; }
    for (int32_t i = 0; i < n; i++) {
        mark[i] = i;
        colcount[i] += 1;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            int32_t r = ri[p];
            while (mark[r] != i) {
                colcount[r] += 1;
                mark[r] = i;
                r = parent[r];
            }
        }
    }
    int64_t nz = 0, fl = 0;
    for (int32_t j = 0; j < n; j++) {
        nz += colcount[j];
        fl += (int64_t)colcount[j] * (int64_t)colcount[j];
    }
    *nnzL = nz;
    *flops = fl;
    free(rp); free(ri); free(iperm); free(anc); free(mark);
    return ORC_OK;
}

/*
 * Column patterns of L: Lp (int64[n+1], from colcount) and Li (row indices,
 * ascending, diagonal first).  Rows are processed in increasing order and
 * row i is appended to every column of its row subtree, so each column comes
 * out sorted.
 */
int orc_pattern(int32_t n, const int64_t *colptr, const int32_t *rowind, const int32_t *perm,
                const int32_t *parent, const int32_t *colcount, int64_t *Lp, int32_t *Li)
{
    int32_t *iperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!iperm || !mark || !pos) { free(iperm); free(mark); free(pos); return ORC_ENOMEM; }
    if (invert_perm(n, perm, iperm)) { free(iperm); free(mark); free(pos); return ORC_EINVAL; }
    int64_t *rp = NULL;
    int32_t *ri = NULL;
    int rc = build_row_lists(n, colptr, rowind, iperm, &rp, &ri);
    if (rc) { free(iperm); free(mark); free(pos); return rc; }
    Lp[0] = 0;
    for (int32_t j = 0; j < n; j++) Lp[j + 1] = Lp[j] + colcount[j];
    for (int32_t j = 0; j < n; j++) { pos[j] = Lp[j]; mark[j] = -1; }
    for (int32_t i = 0; i < n; i++) {
        mark[i] = i;
        Li[pos[i]++] = i;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            int32_t r = ri[p];
            while (mark[r] != i) {
                Li[pos[r]++] = i;
                mark[r] = i;
                r = parent[r];
            }
        }
    }
    for (int32_t j = 0; j < n; j++) {
        if (pos[j] != Lp[j + 1]) { rc = ORC_EINVAL; break; }
    }
    free(rp); free(ri); free(iperm); free(mark); free(pos);
    return rc;
}

/*
 * Left-looking numeric factorization of C = P A P^T into L (pattern Lp, Li
 * from orc_pattern, values into Lx).  Only the first ncols columns are
 * computed (ncols = n for the whole factor); columns j < ncols are exact
 * because column j depends only on columns k < j.
 *
 * For column j: w = C(j:n, j); for every k < j with l_jk != 0,
 * w(rows of column k at or below j) -= l_jk * L(those rows, k);
 * l_jj = sqrt(w_j) (fails unless w_j > 0), l_ij = w_i / l_jj.
 * The columns k with l_jk != 0 are found with one cursor per column (its
 * next row at or below the current j) and one linked list per row.
 */
int orc_factor(int32_t n, const int64_t *colptr, const int32_t *rowind, const double *values,
               const int32_t *perm, const int64_t *Lp, const int32_t *Li, double *Lx,
               int32_t ncols, int32_t *bad_col)
{
    *bad_col = -1;
    if (ncols < 0 || ncols > n) return ORC_EINVAL;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *iperm = (int32_t *)malloc(sizeof(int32_t) * nn);
    int64_t *cp = (int64_t *)calloc(nn + 1, sizeof(int64_t));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * nn);
    int32_t *head = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * nn);
    double *w = (double *)calloc(nn, sizeof(double));
    if (!iperm || !cp || !cur || !head || !next || !w) {
        free(iperm); free(cp); free(cur); free(head); free(next); free(w);
        return ORC_ENOMEM;
    }
    if (invert_perm(n, perm, iperm)) {
        free(iperm); free(cp); free(cur); free(head); free(next); free(w);
        return ORC_EINVAL;
    }
    /* lower CSC of C with values: column lo holds (hi, value) */
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int32_t a = iperm[rowind[p]], b = iperm[j];
            cp[(a < b ? a : b) + 1]++;
        }
    for (int32_t j = 0; j < n; j++) cp[j + 1] += cp[j];
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cp[n] > 0 ? cp[n] : 1));
    double *cx = (double *)malloc(sizeof(double) * (size_t)(cp[n] > 0 ? cp[n] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (nn + 1));
    if (!ci || !cx || !fill) {
        free(iperm); free(cp); free(cur); free(head); free(next); free(w); free(ci); free(cx); free(fill);
        return ORC_ENOMEM;
    }
    memcpy(fill, cp, sizeof(int64_t) * (nn + 1));
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int32_t a = iperm[rowind[p]], b = iperm[j];
            int32_t lo = a < b ? a : b, hi = a < b ? b : a;
            ci[fill[lo]] = hi;
            cx[fill[lo]] = values[p];
            fill[lo]++;
        }
    free(fill);

    for (int32_t j = 0; j < n; j++) head[j] = -1;
    int rc = ORC_OK;
    for (int32_t j = 0; j < ncols; j++) {
        for (int64_t p = cp[j]; p < cp[j + 1]; p++) w[ci[p]] += cx[p];
        /* every column k with l_jk != 0 sits in list j */
        int32_t k = head[j];
        head[j] = -1;
        while (k != -1) {
            int32_t knext = next[k];
            int64_t q = cur[k];              /* Li[q] == j */
            double ljk = Lx[q];
            for (int64_t t = q; t < Lp[k + 1]; t++) w[Li[t]] -= ljk * Lx[t];
            cur[k] = q + 1;
            if (q + 1 < Lp[k + 1]) {
                int32_t r = Li[q + 1];
                next[k] = head[r];
                head[r] = k;
            }
            k = knext;
        }
        double d = w[j];
        if (!(d > 0.0)) {        /* also catches NaN */
            *bad_col = j;
            rc = ORC_ENOTSPD;
            break;
        }
        double ljj = sqrt(d);
        Lx[Lp[j]] = ljj;
        w[j] = 0.0;
        for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; p++) {
            Lx[p] = w[Li[p]] / ljj;
            w[Li[p]] = 0.0;
        }
        cur[j] = Lp[j] + 1;
        if (Lp[j] + 1 < Lp[j + 1]) {
            int32_t r = Li[Lp[j] + 1];
            next[j] = head[r];
            head[r] = j;
        }
    }
    free(iperm); free(cp); free(cur); free(head); free(next); free(w); free(ci); free(cx);
    return rc;
}

/*
 * Triangular solves with the factor, one right-hand side column at a time.
 *   part 0: X = P^T L^-T L^-1 P B    (the solve with A)
 *   part 1: X = L^-1 P B             (result in pivot order)
 *   part 2: X = P^T L^-T B           (input in pivot order)
 * B and X are column-major n x nrhs with leading dimension ld; they may alias.
 */
int orc_solve(int32_t n, const int32_t *perm, const int64_t *Lp, const int32_t *Li, const double *Lx,
              int32_t part, int32_t nrhs, const double *B, double *X, int64_t ld)
{
    if (part < 0 || part > 2 || ld < n) return ORC_EINVAL;
    double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!y) return ORC_ENOMEM;
    for (int32_t c = 0; c < nrhs; c++) {
        const double *b = B + (size_t)c * (size_t)ld;
        double *x = X + (size_t)c * (size_t)ld;
        if (part == 2) {
            for (int32_t k = 0; k < n; k++) y[k] = b[k];
        } else {
            for (int32_t k = 0; k < n; k++) y[k] = b[perm[k]];
        }
        if (part != 2) {
            /* forward: L y = y, column by column */
            for (int32_t j = 0; j < n; j++) {
                y[j] /= Lx[Lp[j]];
                double yj = y[j];
                for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; p++) y[Li[p]] -= Lx[p] * yj;
            }
        }
        if (part != 1) {
            /* backward: L^T y = y, one dot product per column */
            for (int32_t j = n - 1; j >= 0; j--) {
                double s = y[j];
                for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; p++) s -= Lx[p] * y[Li[p]];
                y[j] = s / Lx[Lp[j]];
            }
        }
        if (part == 1) {
            for (int32_t k = 0; k < n; k++) x[k] = y[k];
        } else {
            for (int32_t k = 0; k < n; k++) x[perm[k]] = y[k];
        }
    }
    free(y);
    return ORC_OK;
}

/*
 * Products with the factor itself (the operators of P A P^T = L L^T, reused
 * like the solves; x = P^T L z with white noise z has covariance A):
 *   part 1: X = P^T L B     (input in pivot order)
 *   part 2: X = L^T P B     (result in pivot order)
 * so part 1 applied to the result of part 2 gives P^T L L^T P B = A B.
 * B and X are column-major n x nrhs with leading dimension ld; they may alias.
 */
int orc_apply(int32_t n, const int32_t *perm, const int64_t *Lp, const int32_t *Li, const double *Lx,
              int32_t part, int32_t nrhs, const double *B, double *X, int64_t ld)
{
    if (part < 1 || part > 2 || ld < n) return ORC_EINVAL;
    double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *z = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!y || !z) { free(y); free(z); return ORC_ENOMEM; }
    for (int32_t c = 0; c < nrhs; c++) {
        const double *b = B + (size_t)c * (size_t)ld;
        double *x = X + (size_t)c * (size_t)ld;
        if (part == 1) {
            /* z = L y, column by column: column j of L scaled by y_j */
            for (int32_t k = 0; k < n; k++) { y[k] = b[k]; z[k] = 0.0; }
            for (int32_t j = 0; j < n; j++)
                for (int64_t p = Lp[j]; p < Lp[j + 1]; p++) z[Li[p]] += Lx[p] * y[j];
            for (int32_t k = 0; k < n; k++) x[perm[k]] = z[k];
        } else {
            /* z = L^T y: entry j is column j of L dotted with y */
            for (int32_t k = 0; k < n; k++) y[k] = b[perm[k]];
            for (int32_t j = 0; j < n; j++) {
                double s = 0.0;
                for (int64_t p = Lp[j]; p < Lp[j + 1]; p++) s += Lx[p] * y[Li[p]];
                z[j] = s;
            }
            for (int32_t k = 0; k < n; k++) x[k] = z[k];
        }
    }
    free(y);
    free(z);
    return ORC_OK;
}

/*
 * Y = A X for the full symmetric A given by its lower CSC, in original order.
 */
int orc_symv(int32_t n, const int64_t *colptr, const int32_t *rowind, const double *values,
             int32_t nrhs, const double *X, double *Y, int64_t ld)
{
    if (ld < n) return ORC_EINVAL;
    for (int32_t c = 0; c < nrhs; c++) {
        const double *x = X + (size_t)c * (size_t)ld;
        double *y = Y + (size_t)c * (size_t)ld;
        for (int32_t i = 0; i < n; i++) y[i] = 0.0;
        for (int32_t j = 0; j < n; j++) {
            for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
                int32_t i = rowind[p];
                y[i] += values[p] * x[j];
                if (i != j) y[j] += values[p] * x[i];
            }
        }
    }
    return ORC_OK;
}

/*
 * Gradient of a loss through x = A^-1 b with respect to the stored lower
 * entries of A, given lambda = A^-1 (dloss/dx) and x: an off-diagonal stored
 * entry a_ij (i > j) stands for both a_ij and a_ji, so its gradient is
 * -(lambda_i x_j + lambda_j x_i); a diagonal entry gets -lambda_i x_i.
 */
int orc_grad(int32_t n, const int64_t *colptr, const int32_t *rowind, const double *lam,
             const double *x, double *gA)
{
    for (int32_t j = 0; j < n; j++) {
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int32_t i = rowind[p];
            if (i == j) gA[p] = -lam[i] * x[i];
            else gA[p] = -(lam[i] * x[j] + lam[j] * x[i]);
        }
    }
    return ORC_OK;
}

/*
 * Nested dissection block structure.  Node t of the separator tree is
 * tree[6t .. 6t+5] = (lo, mid, sep, hi, child1, child2) in pivot positions:
 * the subtree's vertices are perm[lo:hi], V1 = perm[lo:mid],
 * V2 = perm[mid:sep], S = perm[sep:hi]; child1/child2 are the node indices
 * for V1 and V2 (-1 for none).  A leaf (no further split) has mid = -1 and
 * sep = lo.  The root is node 0 and covers all n positions.
 * Checks: perm is a bijection; each child's range equals its V1/V2 range;
 * no stored entry of A joins a vertex of V1 with a vertex of V2.
 * Returns the number of violations found (0 = valid), or a negative code.
 */
int64_t orc_check_nd(int32_t n, const int64_t *colptr, const int32_t *rowind, const int32_t *perm,
                     int32_t nnodes, const int32_t *tree)
{
    if (nnodes < 1) return ORC_EINVAL;
    int32_t *iperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!iperm) return ORC_ENOMEM;
    if (invert_perm(n, perm, iperm)) { free(iperm); return ORC_EINVAL; }
    int64_t bad = 0;
    const int32_t *root = tree;
    if (root[0] != 0 || root[3] != n) bad++;
    for (int32_t t = 0; t < nnodes; t++) {
        const int32_t *nd = tree + 6 * (size_t)t;
        int32_t lo = nd[0], mid = nd[1], sep = nd[2], hi = nd[3];
        if (!(0 <= lo && lo <= sep && sep <= hi && hi <= n)) { bad++; continue; }
        if (mid >= 0) {
            if (!(lo <= mid && mid <= sep)) { bad++; continue; }
            int32_t c1 = nd[4], c2 = nd[5];
            if (c1 >= 0) {
                if (c1 >= nnodes || tree[6 * (size_t)c1] != lo || tree[6 * (size_t)c1 + 3] != mid) bad++;
            } else if (mid != lo) bad++;
            if (c2 >= 0) {
                if (c2 >= nnodes || tree[6 * (size_t)c2] != mid || tree[6 * (size_t)c2 + 3] != sep) bad++;
            } else if (sep != mid) bad++;
        }
    }
    /* walk every edge down from the root */
    for (int32_t j = 0; j < n; j++) {
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int32_t i = rowind[p];
            if (i == j) continue;
            int32_t a = iperm[i], b = iperm[j];
            int32_t t = 0;
            for (int guard = 0; guard <= nnodes; guard++) {
                const int32_t *nd = tree + 6 * (size_t)t;
                int32_t lo = nd[0], mid = nd[1], sep = nd[2];
                if (mid < 0) break;                       /* leaf: no constraint */
                if (a < lo || b < lo || a >= sep || b >= sep) break;   /* one is in S (or outside) */
                int ain1 = a < mid, bin1 = b < mid;
                if (ain1 != bin1) { bad++; break; }
                t = ain1 ? nd[4] : nd[5];
                if (t < 0) break;
            }
        }
    }
    free(iperm);
    return bad;
}

/* ------------------------------------------------------------------ LU */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Left-looking sparse LU without pivoting of C = P A P^T for a matrix A with
 * a symmetric pattern (Section 5.1, eq:PCM2: the PCM system matrix; Section
 * 6.1 factors it by LU on the nested dissection ordering).  A is given by its
 * stored lower pattern (colptr, rowind) with two values per stored entry
 * (r, c), r >= c: lval = A[r][c] and uval = A[c][r] (equal on the diagonal;
 * uval of a diagonal entry is not read).
 *
 * Column j of the factors is the sparse triangular solve L(0:j,0:j) u = C(0:j, j)
 * followed by l = (C(j+1:n, j) - L(j+1:n, 0:j) u) / u_jj: with w = C(:, j)
 * scattered into a dense vector, for every k < j with u_kj != 0 in ascending
 * order (each u_kj is final once the columns before k have been applied),
 * u_kj = w[k] and w[i] -= l_ik u_kj for the rows i > k of column k of L.  The
 * pattern of column j of U is that of row j of L (symmetric pattern), so the
 * columns k are found with the same per-column "next row" lists as the
 * Cholesky oracle.
 *
 * Output in the pattern (Lp, Li) of the Cholesky factor (orc_pattern):
 * Lx = L with its unit diagonal stored as 1, Ux = U^T (entry q of column k,
 * row Li[q], holds u(k, Li[q]); the diagonal slot holds u_kk).  Only the
 * first ncols columns of both are computed (the rest untouched).
 */
int orc_lu(int32_t n, const int64_t *colptr, const int32_t *rowind, const double *lval, const double *uval,
           const int32_t *perm, const int64_t *Lp, const int32_t *Li, double *Lx, double *Ux,
           int32_t ncols, int32_t *bad_col)
{
    *bad_col = -1;
    if (ncols < 0 || ncols > n) return ORC_EINVAL;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *iperm = (int32_t *)malloc(sizeof(int32_t) * nn);
    int64_t *cp = (int64_t *)calloc(nn + 1, sizeof(int64_t));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * nn);
    int32_t *head = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *ks = (int32_t *)malloc(sizeof(int32_t) * nn);
    double *w = (double *)calloc(nn, sizeof(double));
    int64_t nnz = colptr[n];
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * nnz > 0 ? 2 * nnz : 1));
    double *cx = (double *)malloc(sizeof(double) * (size_t)(2 * nnz > 0 ? 2 * nnz : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (nn + 1));
    int rc = ORC_OK;
    if (!iperm || !cp || !cur || !head || !next || !ks || !w || !ci || !cx || !fill) {
        rc = ORC_ENOMEM;
        goto done;
    }
    if (invert_perm(n, perm, iperm)) { rc = ORC_EINVAL; goto done; }
    /* full CSC of C (both triangles): entry (r, c) of A lands at (iperm[r], iperm[c]) */
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int32_t r = rowind[p];
            cp[iperm[j] + 1]++;                 /* C(iperm[r], iperm[j]) = A[r][j] */
            if (r != j) cp[iperm[r] + 1]++;     /* C(iperm[j], iperm[r]) = A[j][r] */
        }
    for (int32_t j = 0; j < n; j++) cp[j + 1] += cp[j];
    memcpy(fill, cp, sizeof(int64_t) * (nn + 1));
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int32_t r = rowind[p];
            int32_t a = iperm[r], b = iperm[j];
            ci[fill[b]] = a;
            cx[fill[b]++] = lval[p];
            if (r != j) {
                ci[fill[a]] = b;
                cx[fill[a]++] = uval[p];
            }
        }
    for (int32_t j = 0; j < n; j++) head[j] = -1;
    for (int32_t j = 0; j < ncols; j++) {
        for (int64_t p = cp[j]; p < cp[j + 1]; p++) w[ci[p]] += cx[p];
        /* the columns k < j with l_jk != 0 (= the rows of column j of U) */
        int32_t nk = 0;
        for (int32_t k = head[j]; k != -1; k = next[k]) ks[nk++] = k;
        head[j] = -1;
        qsort(ks, (size_t)nk, sizeof(int32_t), cmp_i32);
        for (int32_t t = 0; t < nk; t++) {
            int32_t k = ks[t];
            int64_t q = cur[k];                 /* Li[q] == j */
            double ukj = w[k];
            Ux[q] = ukj;                        /* u(k, j) in column k of U^T */
            w[k] = 0.0;
            for (int64_t r = Lp[k] + 1; r < Lp[k + 1]; r++) w[Li[r]] -= Lx[r] * ukj;
            cur[k] = q + 1;
            if (q + 1 < Lp[k + 1]) {
                int32_t r = Li[q + 1];
                next[k] = head[r];
                head[r] = k;
            }
        }
        double d = w[j];
        if (d == 0.0 || !isfinite(d)) {
            *bad_col = j;
            rc = ORC_ESINGULAR;
            break;
        }
        Ux[Lp[j]] = d;
        Lx[Lp[j]] = 1.0;
        w[j] = 0.0;
        for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; p++) {
            Lx[p] = w[Li[p]] / d;
            w[Li[p]] = 0.0;
        }
        cur[j] = Lp[j] + 1;
        if (Lp[j] + 1 < Lp[j + 1]) {
            int32_t r = Li[Lp[j] + 1];
            next[j] = head[r];
            head[r] = j;
        }
    }
done:
    free(iperm); free(cp); free(cur); free(head); free(next); free(ks); free(w); free(ci); free(cx); free(fill);
    return rc;
}

/*
 * x = P^T U^-1 L^-1 P b with the factors of orc_lu (part 0); part 1 stops
 * after the forward substitution (L^-1 P b, pivot order), part 2 does only
 * the backward one (P^T U^-1 b, input in pivot order).  Forward: column
 * oriented with the unit lower L; backward: u_jj z_j = y_j - sum_{i>j}
 * u(j, i) z_i, the sum running down column j of U^T.
 */
int orc_lu_solve(int32_t n, const int32_t *perm, const int64_t *Lp, const int32_t *Li, const double *Lx,
                 const double *Ux, int32_t part, int32_t nrhs, const double *B, double *X, int64_t ld)
{
    if (part < 0 || part > 2 || ld < n) return ORC_EINVAL;
    double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!y) return ORC_ENOMEM;
    for (int32_t c = 0; c < nrhs; c++) {
        const double *b = B + (size_t)c * (size_t)ld;
        double *x = X + (size_t)c * (size_t)ld;
        for (int32_t k = 0; k < n; k++) y[k] = part == 2 ? b[k] : b[perm[k]];
        if (part != 2)
            for (int32_t j = 0; j < n; j++) {
                double yj = y[j];
                for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; p++) y[Li[p]] -= Lx[p] * yj;
            }
        if (part != 1)
            for (int32_t j = n - 1; j >= 0; j--) {
                double s = y[j];
                for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; p++) s -= Ux[p] * y[Li[p]];
                y[j] = s / Ux[Lp[j]];
            }
        for (int32_t k = 0; k < n; k++) {
            if (part == 1) x[k] = y[k];
            else x[perm[k]] = y[k];
        }
    }
    free(y);
    return ORC_OK;
}

/*
 * Y = A X for the nonsymmetric A given by its stored lower pattern with the
 * two values of orc_lu (lval below and on the diagonal, uval above), in the
 * original order.
 */
int orc_gemv(int32_t n, const int64_t *colptr, const int32_t *rowind, const double *lval, const double *uval,
             int32_t nrhs, const double *X, double *Y, int64_t ld)
{
    if (ld < n) return ORC_EINVAL;
    for (int32_t c = 0; c < nrhs; c++) {
        const double *x = X + (size_t)c * (size_t)ld;
        double *y = Y + (size_t)c * (size_t)ld;
        for (int32_t i = 0; i < n; i++) y[i] = 0.0;
        for (int32_t j = 0; j < n; j++)
            for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
                int32_t i = rowind[p];
                y[i] += lval[p] * x[j];
                if (i != j) y[j] += uval[p] * x[i];
            }
    }
    return ORC_OK;
}
