/*
 * ORACLE -- test infrastructure only.  Nothing in the product links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or table with the GPU library.
 *
 * A plain, serial, FP64 left-looking Gilbert-Peierls sparse LU with threshold
 * partial pivoting, written from the paper's description:
 *
 *   - Alg. 1 (Gilbert-Peierls): for every column k, find the topological order of
 *     the fill pattern of A(:,k) by depth-first search on the graph of L, apply the
 *     sparse triangular updates x -= L(:,j) x_j for j in that order, select the
 *     pivot from the updated column, and copy it into L and U.
 *   - Sec. II / III-A (BTF): only the diagonal blocks of the permuted matrix are
 *     factored; the off-diagonal blocks are kept as they are for the solve.
 *   - Sec. III-C (fine ND): pivoting is limited to the rows of the column's own
 *     nested-dissection node; rows of ancestor separators are computed into L but
 *     never chosen as pivots for that column.
 *   - Sec. V-F (transient sequence): the symbolic analysis is reused for new
 *     values; the refactor below replays the factorization with the stored pivots.
 *
 * The permuted matrix is R = A(prow, qcol).  Candidate groups are contiguous
 * ranges of R's index space (grpptr), nested inside BTF blocks (blkptr).  For a
 * column k in group [g0, g1) the candidates are the non-pivotal rows i of the
 * updated column with g0 <= i < g1.  With m the largest candidate magnitude:
 *   if diag_pref and row k is a candidate and |x_k| >= tau*m, the pivot is k;
 *   otherwise it is the smallest candidate index attaining m.
 * A column with no candidate or m == 0 is numerically singular.
 *
 * Arithmetic: every update is x[r] = x[r] - (l * xj) with separate rounding (the
 * file is compiled with -ffp-contract=off), and L(i,k) = x_i / x_p (IEEE division).
 * The update order is the DFS reverse postorder (order = 0), or ascending pivot
 * index (order = 1), which is also a topological order because every edge of the
 * graph of L runs from a lower to a higher pivot index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_INVALID (-1)
#define OR_ERR_NUM_SINGULAR (-3)
#define OR_ERR_OOM (-4)
#define OR_REFACTOR_FAIL (-7)

typedef struct {
    int n;
    /* factors in pivot order: L strictly lower (unit diagonal implicit), U upper with diagonal */
    int64_t *Lp; int32_t *Li; double *Lx;
    int64_t *Up; int32_t *Ui; double *Ux;
    int32_t *piv;      /* piv[k] = row of R chosen as pivot of column k */
    double *margin;    /* relative decision margin of each column's pivot choice */
    double flops;
    int status;
    int fail_col;
} or_result;

/* growable arrays */
typedef struct { int32_t *i; double *x; int64_t len, cap; } or_buf;

static int buf_push(or_buf *b, int32_t i, double x) {
    if (b->len == b->cap) {
        int64_t nc = b->cap ? 2 * b->cap : 1024;
        int32_t *ni = (int32_t *)realloc(b->i, (size_t)nc * sizeof(int32_t));
        if (!ni) return 0;
        b->i = ni;
        double *nx = (double *)realloc(b->x, (size_t)nc * sizeof(double));
        if (!nx) return 0;
        b->x = nx;
        b->cap = nc;
    }
    b->i[b->len] = i; b->x[b->len] = x; b->len++;
    return 1;
}

static int cmp_pair_idx(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

typedef struct { int32_t key; double val; } kv;
static int cmp_kv(const void *a, const void *b) {
    int32_t x = ((const kv *)a)->key, y = ((const kv *)b)->key;
    return (x > y) - (x < y);
}

void or_free(or_result *r) {
    if (!r) return;
    free(r->Lp); free(r->Li); free(r->Lx);
    free(r->Up); free(r->Ui); free(r->Ux);
    free(r->piv); free(r->margin);
    free(r);
}

/*
 * Factor (forced_piv == NULL) or refactor (forced_piv = pivots of an earlier
 * factorization with the same pattern).  A refactor takes the forced pivot and
 * fails with OR_REFACTOR_FAIL at the first column where x_p == 0 or
 * |x_p| < tau * (largest candidate magnitude).
 */
or_result *or_factor(int n, const int32_t *Ap, const int32_t *Ai, const double *Ax,
                     const int32_t *prow, const int32_t *qcol,
                     int nblk, const int32_t *blkptr, int ngrp, const int32_t *grpptr,
                     double tau, int diag_pref, int order, const int32_t *forced_piv)
{
    or_result *res = (or_result *)calloc(1, sizeof(or_result));
    if (!res) return NULL;
    res->n = n;
    res->fail_col = -1;
    res->status = OR_OK;

    int32_t *pinvrow = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));   /* A row -> R row */
    int32_t *pinv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));      /* R row -> column it pivots, -1 */
    int32_t *grp_lo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));    /* column -> group start */
    int32_t *grp_hi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *blk_lo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *blk_hi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *spos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *pattern = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *pivlist = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * 2);
    double *x = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    /* L during the factorization: columns in R-row space */
    int64_t *Lcol = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    or_buf Lb = {0}, Ub = {0};
    int64_t *Ucol = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    res->piv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    res->margin = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!pinvrow || !pinv || !grp_lo || !grp_hi || !blk_lo || !blk_hi || !mark || !stack || !spos ||
        !pattern || !pivlist || !x || !Lcol || !Ucol || !res->piv || !res->margin) {
        res->status = OR_ERR_OOM;
        goto done;
    }

    /* validate the orderings */
    for (int i = 0; i < n; i++) pinvrow[i] = -1;
    for (int i = 0; i < n; i++) {
        if (prow[i] < 0 || prow[i] >= n || pinvrow[prow[i]] >= 0) { res->status = OR_ERR_INVALID; goto done; }
        pinvrow[prow[i]] = i;
    }
    for (int i = 0; i < n; i++) mark[i] = -1;
    for (int k = 0; k < n; k++) {
        if (qcol[k] < 0 || qcol[k] >= n || mark[qcol[k]] >= 0) { res->status = OR_ERR_INVALID; goto done; }
        mark[qcol[k]] = k;
    }
    if (blkptr[0] != 0 || blkptr[nblk] != n || grpptr[0] != 0 || grpptr[ngrp] != n) {
        res->status = OR_ERR_INVALID; goto done;
    }
    for (int b = 0; b < nblk; b++) {
        if (blkptr[b + 1] <= blkptr[b]) { res->status = OR_ERR_INVALID; goto done; }
        for (int k = blkptr[b]; k < blkptr[b + 1]; k++) { blk_lo[k] = blkptr[b]; blk_hi[k] = blkptr[b + 1]; }
    }
    for (int g = 0; g < ngrp; g++) {
        if (grpptr[g + 1] <= grpptr[g]) { res->status = OR_ERR_INVALID; goto done; }
        for (int k = grpptr[g]; k < grpptr[g + 1]; k++) {
            grp_lo[k] = grpptr[g]; grp_hi[k] = grpptr[g + 1];
            if (grp_lo[k] < blk_lo[k] || grp_hi[k] > blk_hi[k]) { res->status = OR_ERR_INVALID; goto done; }
        }
    }

    for (int i = 0; i < n; i++) { pinv[i] = -1; mark[i] = -1; }
    Lcol[0] = 0; Ucol[0] = 0;
    double flops = 0.0;

    for (int k = 0; k < n; k++) {
        const int b0 = blk_lo[k], b1 = blk_hi[k];
        const int g0 = grp_lo[k], g1 = grp_hi[k];
        const int acol = qcol[k];
        /* rows of R(:,k) inside the diagonal block, ascending */
        int top = n;  /* pattern[top..n-1] holds the topological order */
        int nA = 0;
        for (int32_t p = Ap[acol]; p < Ap[acol + 1]; p++) {
            int i = pinvrow[Ai[p]];
            if (i >= b1) { res->status = OR_ERR_INVALID; res->fail_col = k; goto done; } /* below the block: not BTF */
            if (i < b0) continue;                                                        /* off-diagonal block */
            pivlist[nA++] = i;
        }
        qsort(pivlist, (size_t)nA, sizeof(int32_t), cmp_pair_idx);
        /* depth-first search from every row of the column, in ascending order */
        for (int a = 0; a < nA; a++) {
            int start = pivlist[a];
            if (mark[start] == k) continue;
            int head = 0;
            stack[0] = start;
            mark[start] = k;
            spos[start] = (pinv[start] >= 0) ? Lcol[pinv[start]] : -1;
            while (head >= 0) {
                int i = stack[head];
                int j = pinv[i];
                int descended = 0;
                if (j >= 0) {
                    int64_t end = Lcol[j + 1];
                    for (int64_t p = spos[i]; p < end; p++) {
                        int r = Lb.i[p];
                        if (mark[r] != k) {
                            spos[i] = p + 1;
                            mark[r] = k;
                            spos[r] = (pinv[r] >= 0) ? Lcol[pinv[r]] : -1;
                            stack[++head] = r;
                            descended = 1;
                            break;
                        }
                    }
                }
                if (!descended) {
                    head--;
                    pattern[--top] = i;   /* postorder, stored backwards = reverse postorder */
                }
            }
        }
        /* numeric: x = R(:,k) on the pattern, then the sparse triangular solve */
        for (int t = top; t < n; t++) x[pattern[t]] = 0.0;
        for (int32_t p = Ap[acol]; p < Ap[acol + 1]; p++) {
            int i = pinvrow[Ai[p]];
            if (i >= b0 && i < b1) x[i] = Ax[p];
        }
        int npiv = 0;
        if (order == 0) {
            for (int t = top; t < n; t++) {
                int i = pattern[t];
                if (pinv[i] >= 0) pivlist[npiv++] = i;
            }
        } else {
            /* ascending pivot index: sort (pinv, row) pairs */
            for (int t = top; t < n; t++) {
                int i = pattern[t];
                if (pinv[i] >= 0) { pivlist[2 * npiv] = pinv[i]; pivlist[2 * npiv + 1] = i; npiv++; }
            }
            qsort(pivlist, (size_t)npiv, 2 * sizeof(int32_t), cmp_pair_idx);
            for (int q = 0; q < npiv; q++) pivlist[q] = pivlist[2 * q + 1];
        }
        for (int q = 0; q < npiv; q++) {
            int i = pivlist[q];
            int j = pinv[i];
            double xj = x[i];
            for (int64_t p = Lcol[j]; p < Lcol[j + 1]; p++) {
                double prod = Lb.x[p] * xj;
                x[Lb.i[p]] = x[Lb.i[p]] - prod;
            }
            flops += 2.0 * (double)(Lcol[j + 1] - Lcol[j]);
        }
        /* pivot selection among the candidates of the column's group */
        double m = 0.0;
        int have_cand = 0;
        for (int t = top; t < n; t++) {
            int i = pattern[t];
            if (pinv[i] >= 0 || i < g0 || i >= g1) continue;
            have_cand = 1;
            if (fabs(x[i]) > m) m = fabs(x[i]);
        }
        /* smallest candidate index attaining m */
        int argmax = -1;
        for (int t = top; t < n; t++) {
            int i = pattern[t];
            if (pinv[i] >= 0 || i < g0 || i >= g1) continue;
            if (fabs(x[i]) == m && (argmax < 0 || i < argmax)) argmax = i;
        }
        int diag_cand = (mark[k] == k && pinv[k] < 0 && k >= g0 && k < g1);
        int p;
        if (forced_piv) {
            p = forced_piv[k];
            int ok = have_cand && p >= g0 && p < g1 && mark[p] == k && pinv[p] < 0 && x[p] != 0.0 &&
                     fabs(x[p]) >= tau * m;
            if (!ok) { res->status = OR_REFACTOR_FAIL; res->fail_col = k; goto done; }
        } else {
            if (!have_cand || !(m > 0.0)) { res->status = OR_ERR_NUM_SINGULAR; res->fail_col = k; goto done; }
            if (diag_pref && diag_cand && fabs(x[k]) >= tau * m) p = k;
            else p = argmax;
        }
        /* decision margin (relative to m) of the choice just made.  For tau <= 1 the
         * diagonal test |x_k| >= tau * m passes exactly when |x_k| >= tau * m_o, with
         * m_o the largest candidate magnitude other than row k (row k itself can never
         * fail against its own magnitude), so its margin is measured against m_o; a
         * diagonal that is the only candidate is decided outright.  The argmax choice,
         * when it matters, is measured by the gap to the runner-up. */
        {
            double mu = INFINITY;
            if (m > 0.0) {
                if (diag_pref && diag_cand) {
                    double mo = -1.0;
                    for (int t = top; t < n; t++) {
                        int i = pattern[t];
                        if (pinv[i] >= 0 || i < g0 || i >= g1 || i == k) continue;
                        if (fabs(x[i]) > mo) mo = fabs(x[i]);
                    }
                    if (mo >= 0.0) mu = fabs(fabs(x[k]) - tau * mo) / m;
                }
                if (!(diag_pref && diag_cand && fabs(x[k]) >= tau * m)) {
                    double m2 = 0.0; int any2 = 0;
                    for (int t = top; t < n; t++) {
                        int i = pattern[t];
                        if (pinv[i] >= 0 || i < g0 || i >= g1 || i == argmax) continue;
                        any2 = 1;
                        if (fabs(x[i]) > m2) m2 = fabs(x[i]);
                    }
                    if (any2) { double g = (m - m2) / m; if (g < mu) mu = g; }
                }
            }
            res->margin[k] = mu;
        }
        res->piv[k] = p;
        /* store U(:,k) (pivot-space rows), then L(:,k) (R rows, ascending) */
        double xp = x[p];
        for (int t = top; t < n; t++) {
            int i = pattern[t];
            if (pinv[i] >= 0) { if (!buf_push(&Ub, pinv[i], x[i])) { res->status = OR_ERR_OOM; goto done; } }
        }
        if (!buf_push(&Ub, k, xp)) { res->status = OR_ERR_OOM; goto done; }
        Ucol[k + 1] = Ub.len;
        int64_t lstart = Lb.len;
        for (int t = top; t < n; t++) {
            int i = pattern[t];
            if (pinv[i] < 0 && i != p) {
                double l = x[i] / xp;
                if (!buf_push(&Lb, i, l)) { res->status = OR_ERR_OOM; goto done; }
            }
        }
        /* ascending R-row order inside the column */
        {
            int64_t cnt = Lb.len - lstart;
            if (cnt > 1) {
                kv *tmp = (kv *)malloc(sizeof(kv) * (size_t)cnt);
                if (!tmp) { res->status = OR_ERR_OOM; goto done; }
                for (int64_t q = 0; q < cnt; q++) { tmp[q].key = Lb.i[lstart + q]; tmp[q].val = Lb.x[lstart + q]; }
                qsort(tmp, (size_t)cnt, sizeof(kv), cmp_kv);
                for (int64_t q = 0; q < cnt; q++) { Lb.i[lstart + q] = tmp[q].key; Lb.x[lstart + q] = tmp[q].val; }
                free(tmp);
            }
            flops += (double)cnt;
        }
        Lcol[k + 1] = Lb.len;
        pinv[p] = k;
    }
    res->flops = flops;

    /* convert L to pivot order and sort rows inside every column; sort U rows too */
    res->Lp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    res->Up = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    res->Li = (int32_t *)malloc(sizeof(int32_t) * (size_t)(Lb.len > 0 ? Lb.len : 1));
    res->Lx = (double *)malloc(sizeof(double) * (size_t)(Lb.len > 0 ? Lb.len : 1));
    res->Ui = (int32_t *)malloc(sizeof(int32_t) * (size_t)(Ub.len > 0 ? Ub.len : 1));
    res->Ux = (double *)malloc(sizeof(double) * (size_t)(Ub.len > 0 ? Ub.len : 1));
    if (!res->Lp || !res->Up || !res->Li || !res->Lx || !res->Ui || !res->Ux) { res->status = OR_ERR_OOM; goto done; }
    for (int k = 0; k <= n; k++) { res->Lp[k] = Lcol[k]; res->Up[k] = Ucol[k]; }
    for (int k = 0; k < n; k++) {
        int64_t a = Lcol[k], b = Lcol[k + 1];
        int64_t cnt = b - a;
        kv *tmp = (kv *)malloc(sizeof(kv) * (size_t)(cnt > 0 ? cnt : 1));
        if (!tmp) { res->status = OR_ERR_OOM; goto done; }
        for (int64_t q = 0; q < cnt; q++) { tmp[q].key = pinv[Lb.i[a + q]]; tmp[q].val = Lb.x[a + q]; }
        qsort(tmp, (size_t)cnt, sizeof(kv), cmp_kv);
        for (int64_t q = 0; q < cnt; q++) { res->Li[a + q] = tmp[q].key; res->Lx[a + q] = tmp[q].val; }
        a = Ucol[k]; b = Ucol[k + 1]; cnt = b - a;
        kv *tu = (kv *)realloc(tmp, sizeof(kv) * (size_t)(cnt > 0 ? cnt : 1));
        if (!tu) { free(tmp); res->status = OR_ERR_OOM; goto done; }
        tmp = tu;
        for (int64_t q = 0; q < cnt; q++) { tmp[q].key = Ub.i[a + q]; tmp[q].val = Ub.x[a + q]; }
        qsort(tmp, (size_t)cnt, sizeof(kv), cmp_kv);
        for (int64_t q = 0; q < cnt; q++) { res->Ui[a + q] = tmp[q].key; res->Ux[a + q] = tmp[q].val; }
        free(tmp);
    }

done:
    free(pinvrow); free(pinv); free(grp_lo); free(grp_hi); free(blk_lo); free(blk_hi);
    free(mark); free(stack); free(spos); free(pattern); free(pivlist); free(x);
    free(Lcol); free(Ucol); free(Lb.i); free(Lb.x); free(Ub.i); free(Ub.x);
    return res;
}

int or_status(const or_result *r) { return r->status; }
int or_fail_col(const or_result *r) { return r->fail_col; }
double or_flops(const or_result *r) { return r->flops; }
int64_t or_lnz(const or_result *r) { return r->Lp ? r->Lp[r->n] : 0; }
int64_t or_unz(const or_result *r) { return r->Up ? r->Up[r->n] : 0; }

/* copy the factors out; arrays sized n+1 / lnz / unz / n by the caller */
void or_get(const or_result *r, int64_t *Lp, int32_t *Li, double *Lx, int64_t *Up, int32_t *Ui, double *Ux,
            int32_t *piv, double *margin)
{
    int n = r->n;
    int64_t lnz = or_lnz(r), unz = or_unz(r);
    if (Lp) memcpy(Lp, r->Lp, sizeof(int64_t) * (size_t)(n + 1));
    if (Li) memcpy(Li, r->Li, sizeof(int32_t) * (size_t)lnz);
    if (Lx) memcpy(Lx, r->Lx, sizeof(double) * (size_t)lnz);
    if (Up) memcpy(Up, r->Up, sizeof(int64_t) * (size_t)(n + 1));
    if (Ui) memcpy(Ui, r->Ui, sizeof(int32_t) * (size_t)unz);
    if (Ux) memcpy(Ux, r->Ux, sizeof(double) * (size_t)unz);
    if (piv) memcpy(piv, r->piv, sizeof(int32_t) * (size_t)n);
    if (margin) memcpy(margin, r->margin, sizeof(double) * (size_t)n);
}

/*
 * Solve A X = B for nrhs columns (column-major, leading dimension ldb), in place.
 * With R = A(prow, qcol) = blockdiag(B_b) + strictly-upper off-diagonal blocks and
 * B_b(piv_b, :) = L_b U_b: c = B(prow); for blocks from last to first,
 * r_b = c_b - sum_{c > b} R_bc z_c, then L w = r(piv), U z_b = w; X(qcol) = z.
 */
int or_solve(int n, const int32_t *Ap, const int32_t *Ai, const double *Ax,
             const int32_t *prow, const int32_t *qcol, int nblk, const int32_t *blkptr,
             const or_result *f, int nrhs, double *B, int ldb)
{
    if (f->status != OR_OK) return OR_ERR_INVALID;
    int32_t *pinvrow = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double *c = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *z = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!pinvrow || !c || !z || !w) { free(pinvrow); free(c); free(z); free(w); return OR_ERR_OOM; }
    for (int i = 0; i < n; i++) pinvrow[prow[i]] = i;
    for (int r = 0; r < nrhs; r++) {
        double *bcol = B + (int64_t)r * ldb;
        for (int i = 0; i < n; i++) c[i] = bcol[prow[i]];
        for (int b = nblk - 1; b >= 0; b--) {
            int b0 = blkptr[b], b1 = blkptr[b + 1];
            /* c_b already holds c_b - sum_{c > b} R_bc z_c (scattered after each later block) */
            for (int k = b0; k < b1; k++) w[k] = c[f->piv[k]];
            /* forward: L unit lower, pivot order */
            for (int k = b0; k < b1; k++) {
                double wk = w[k];
                for (int64_t p = f->Lp[k]; p < f->Lp[k + 1]; p++) w[f->Li[p]] = w[f->Li[p]] - f->Lx[p] * wk;
            }
            /* backward: U upper, diagonal last in each column */
            for (int k = b1 - 1; k >= b0; k--) {
                int64_t pd = f->Up[k + 1] - 1;
                double zk = w[k] / f->Ux[pd];
                z[k] = zk;
                for (int64_t p = f->Up[k]; p < pd; p++) w[f->Ui[p]] = w[f->Ui[p]] - f->Ux[p] * zk;
            }
            /* scatter this block's off-diagonal columns into c of earlier blocks */
            for (int k = b0; k < b1; k++) {
                int acol = qcol[k];
                for (int32_t p = Ap[acol]; p < Ap[acol + 1]; p++) {
                    int i = pinvrow[Ai[p]];
                    if (i < b0) c[i] = c[i] - Ax[p] * z[k];
                }
            }
        }
        for (int k = 0; k < n; k++) bcol[qcol[k]] = z[k];
    }
    free(pinvrow); free(c); free(z); free(w);
    return OR_OK;
}
