/*
 * CPU ORACLE -- test infrastructure only.  ILUT(p, tol), the threshold ILU
 * named among the RAS local solvers (the RAS data structure's ilut_p and
 * ilut_tol, default -1 and 1e-3 in the RAS default-parameter figure), for
 * matrices of 3x3 blocks.  Plain serial FP64, sharing no code with the GPU
 * library.
 *
 * The algorithm is Saad's ILUT (Iterative Methods for Sparse Linear
 * Systems, 2nd ed., sec. 10.4) with blocks in place of scalars, block size
 * measured by the squared Frobenius norm |B|^2 = sum of its nine squared
 * entries:
 *   for each row i, ascending:
 *     w = block row i of A;  thr = tol^2 * (sum of |A_ij|^2 over row i)
 *     for k = the present positions of w left of i, in ascending order
 *         (fill created while eliminating is visited in turn):
 *       w_k <- w_k U_kk^-1;  if |w_k|^2 < thr, drop w_k and go on;
 *       else w_j <- w_j - w_k U_kj for every block U_kj of row k right of k
 *         (a position absent from w enters with a zero block);
 *     drop every w_j right of i with |w_j|^2 < thr (the diagonal stays);
 *     keep the p largest left of i and the p largest right of i (ties: the
 *       smaller column first); p < 0 takes, for each side, the number of
 *       blocks of A's row i on that side;
 *     L row i = the kept blocks left of i, U row i = the diagonal and the
 *     kept blocks right of i, U_ii^-1 by LU with partial pivoting.
 * Products of blocks sum their three terms in ascending order; the drop
 * tests compare squared norms, so no square root is taken.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

static void blk_mul(const double *a, const double *b, double *c)   /* c = a b */
{
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            double s = a[3 * p] * b[q];
            s = s + a[3 * p + 1] * b[3 + q];
            s = s + a[3 * p + 2] * b[6 + q];
            c[3 * p + q] = s;
        }
}

static double fro2(const double *a)
{
    double s = 0.0;
    for (int e = 0; e < 9; ++e) s = s + a[e] * a[e];
    return s;
}

typedef struct growing {
    int64_t n, cap;
    int64_t *col;
    double *val;
} growing;

static int grow_push(growing *g, int64_t col, const double *v)
{
    if (g->n == g->cap) {
        int64_t nc = g->cap ? 2 * g->cap : 1024;
        int64_t *c2 = (int64_t *)realloc(g->col, (size_t)nc * sizeof(int64_t));
        if (!c2) return ORC_ERR_OOM;
        g->col = c2;
        double *v2 = (double *)realloc(g->val, (size_t)nc * 9 * sizeof(double));
        if (!v2) return ORC_ERR_OOM;
        g->val = v2;
        g->cap = nc;
    }
    g->col[g->n] = col;
    memcpy(g->val + 9 * g->n, v, 9 * sizeof(double));
    g->n++;
    return ORC_OK;
}

/* the `keep` largest of the candidate columns cand[0..m) by |w|^2 (ties:
 * smaller column first), returned in ascending column order in out */
static int64_t select_largest(const int64_t *cand, int64_t m, const double *w, int64_t keep, int64_t *out)
{
    int64_t nk = 0;
    for (int64_t a = 0; a < m; ++a) {
        const double va = fro2(w + 9 * cand[a]);
        int64_t rank = 0;
        for (int64_t b = 0; b < m; ++b) {
            if (b == a) continue;
            const double vb = fro2(w + 9 * cand[b]);
            if (vb > va || (vb == va && cand[b] < cand[a])) ++rank;
        }
        if (rank < keep) out[nk++] = cand[a];
    }
    /* ascending columns */
    for (int64_t a = 1; a < nk; ++a) {
        const int64_t v = out[a];
        int64_t b = a - 1;
        while (b >= 0 && out[b] > v) {
            out[b + 1] = out[b];
            --b;
        }
        out[b + 1] = v;
    }
    return nk;
}

int orc_ilut(const orc_bcsr *A, int32_t p, double tol, orc_ilu **out, int64_t *bad_cell)
{
    if (!A || !out || !(tol >= 0.0)) return ORC_ERR_ARG;
    if (bad_cell) *bad_cell = -1;
    const int64_t n = A->n;
    double *w = (double *)calloc((size_t)(n > 0 ? n : 1) * 9, sizeof(double));
    char *present = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t *touched = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *cand = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *kept = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    double *dinv = (double *)malloc((size_t)(n > 0 ? n : 1) * 9 * sizeof(double));
    int64_t *rowptr = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t *uptr = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));   /* U rows (diagonal first) */
    growing L = {0, 0, NULL, NULL}, U = {0, 0, NULL, NULL};
    int rc = (w && present && touched && cand && kept && dinv && rowptr && uptr) ? ORC_OK : ORC_ERR_OOM;
    int64_t *lstart = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    if (!lstart) rc = ORC_ERR_OOM;
    for (int64_t i = 0; i < n && rc == ORC_OK; ++i) {
        int64_t nt = 0, nla = 0, nua = 0, lo = i;
        double nrm2 = 0.0;
        for (int64_t q = A->rowptr[i]; q < A->rowptr[i + 1]; ++q) {
            const int64_t j = A->col[q];
            memcpy(w + 9 * j, A->val + 9 * q, 9 * sizeof(double));
            present[j] = 1;
            touched[nt++] = j;
            nrm2 = nrm2 + fro2(A->val + 9 * q);
            if (j < i) ++nla;
            if (j > i) ++nua;
            if (j < lo) lo = j;
        }
        if (!present[i]) {
            rc = ORC_ERR_ZERO_PIVOT;
            if (bad_cell) *bad_cell = i;
            break;
        }
        const double thr = (tol * tol) * nrm2;
        /* elimination: the present positions left of i in ascending order */
        for (int64_t k = lo; k < i; ++k) {
            if (!present[k]) continue;
            double wk[9];
            blk_mul(w + 9 * k, dinv + 9 * k, wk);
            if (fro2(wk) < thr) {
                present[k] = 0;
                continue;
            }
            memcpy(w + 9 * k, wk, sizeof(wk));
            for (int64_t q = uptr[k] + 1; q < uptr[k + 1]; ++q) {
                const int64_t j = U.col[q];
                if (!present[j]) {
                    present[j] = 1;
                    memset(w + 9 * j, 0, 9 * sizeof(double));
                    touched[nt++] = j;
                }
                double prod[9];
                blk_mul(wk, U.val + 9 * q, prod);
                for (int e = 0; e < 9; ++e) w[9 * j + e] = w[9 * j + e] - prod[e];
            }
        }
        /* L: the surviving positions left of i */
        int64_t m = 0;
        for (int64_t t = 0; t < nt; ++t)
            if (touched[t] < i && present[touched[t]]) cand[m++] = touched[t];
        int64_t nk = select_largest(cand, m, w, p < 0 ? nla : p, kept);
        lstart[i] = L.n;
        for (int64_t t = 0; t < nk && rc == ORC_OK; ++t) rc = grow_push(&L, kept[t], w + 9 * kept[t]);
        /* U: the diagonal, then the surviving positions right of i */
        m = 0;
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t j = touched[t];
            if (j > i && present[j] && !(fro2(w + 9 * j) < thr)) cand[m++] = j;
        }
        nk = select_largest(cand, m, w, p < 0 ? nua : p, kept);
        uptr[i] = U.n;
        if (rc == ORC_OK) rc = grow_push(&U, i, w + 9 * i);
        for (int64_t t = 0; t < nk && rc == ORC_OK; ++t) rc = grow_push(&U, kept[t], w + 9 * kept[t]);
        uptr[i + 1] = U.n;
        if (rc == ORC_OK && orc_inv3(w + 9 * i, dinv + 9 * i) != ORC_OK) {
            rc = ORC_ERR_ZERO_PIVOT;
            if (bad_cell) *bad_cell = i;
        }
        for (int64_t t = 0; t < nt; ++t) present[touched[t]] = 0;
    }
    if (rc == ORC_OK) lstart[n] = L.n;
    orc_bcsr *LU = NULL;
    if (rc == ORC_OK) {
        LU = orc_bcsr_new(n, L.n + U.n);
        if (!LU) rc = ORC_ERR_OOM;
    }
    if (rc == ORC_OK) {
        int64_t pos = 0;
        for (int64_t i = 0; i < n; ++i) {
            LU->rowptr[i] = pos;
            for (int64_t q = lstart[i]; q < lstart[i + 1]; ++q, ++pos) {
                LU->col[pos] = L.col[q];
                memcpy(LU->val + 9 * pos, L.val + 9 * q, 9 * sizeof(double));
            }
            for (int64_t q = uptr[i]; q < uptr[i + 1]; ++q, ++pos) {
                LU->col[pos] = U.col[q];
                memcpy(LU->val + 9 * pos, U.val + 9 * q, 9 * sizeof(double));
            }
        }
        LU->rowptr[n] = pos;
    }
    free(w); free(present); free(touched); free(cand); free(kept); free(dinv);
    free(rowptr); free(uptr); free(lstart);
    free(L.col); free(L.val); free(U.col); free(U.val);
    if (rc != ORC_OK) {
        orc_bcsr_free(LU);
        return rc;
    }
    return orc_ilu_wrap(LU, out, bad_cell);
}
