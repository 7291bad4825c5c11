/*
 * CPU ORACLE -- test infrastructure only.  The CPR-type two-stage
 * preconditioners of the paper's CPR-like Preconditioners subsection, in the
 * order of its four algorithms (CPR-FP, CPR-PF, CPR-FPF, CPR-FFPF).  Plain
 * serial FP64, sharing no code with the GPU library.
 *
 *  - pressure restriction Pi_r and prolongation Pi_p (same subsection): the
 *    pressure is component 0 of each cell; Pi_p puts a pressure vector into
 *    component 0 and zeros into the others;
 *  - decoupling (the simulator runs name one but the paper does not define
 *    it; three readings): the pressure equation of cell c is w_c^T times
 *    block row c, with
 *      none         w_c = e_0 (A_pp is the pressure-pressure submatrix),
 *      quasi-IMPES  w_c = (1, w1, w2) with w_c^T D_c zero in columns 1 and 2
 *                   (Scheichl, Masson & Wendebourg 2003), D_c = A_cc,
 *      ABF          w_c^T = e_0^T D_c^-1 (alternate block factorisation,
 *                   Bank, Chan, Coughran & Smith 1989);
 *    A_pp(c, n) = w_c^T A_cn e_0 and the restricted residual is w_c^T r_c;
 *  - M_g(A_pp)^-1: one V-cycle of mg.c's aggregation multigrid;
 *  - R(A)^-1: any oracle preconditioner of the whole system (RAS, ILU(0)),
 *    passed in as a function;
 *  - CPR-PF is taken as x = Pi_p M_g^-1 Pi_r f, r = f - A x, x += R^-1 r
 *    (the printed steps overwrite the first x and apply R to f again).
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

struct orc_cpr {
    const orc_bcsr *A;    /* not owned */
    int64_t n;            /* cells */
    int32_t variant, decouple;
    double *w;            /* [n][3] */
    orc_csr *App;
    orc_mg *mg;
    orc_apply_fn R;
    void *Rctx;
    double *r, *t, *q, *e;
};

void orc_cpr_free(orc_cpr *P)
{
    if (!P) return;
    orc_mg_free(P->mg);
    orc_csr_free(P->App);
    free(P->w);
    free(P->r);
    free(P->t);
    free(P->q);
    free(P->e);
    free(P);
}

/* decoupling weights of one cell from its diagonal block d (row-major) */
static int cell_weights(const double *d, int32_t decouple, double *w)
{
    if (decouple == ORC_DECOUPLE_NONE) {
        w[0] = 1.0;
        w[1] = 0.0;
        w[2] = 0.0;
        return ORC_OK;
    }
    if (decouple == ORC_DECOUPLE_QUASI_IMPES) {
        /* w1 d[1][q] + w2 d[2][q] = -d[0][q] for q = 1, 2 (Cramer's rule) */
        const double det = d[4] * d[8] - d[7] * d[5];
        const double scale = fabs(d[4] * d[8]) + fabs(d[7] * d[5]);
        if (!(fabs(det) > 1e-14 * scale) || !(fabs(det) > 1e-300)) return ORC_ERR_ZERO_PIVOT;
        w[0] = 1.0;
        w[1] = (-d[1] * d[8] + d[7] * d[2]) / det;
        w[2] = (-d[4] * d[2] + d[1] * d[5]) / det;
        return ORC_OK;
    }
    if (decouple == ORC_DECOUPLE_ABF) {
        double inv[9];
        const int rc = orc_inv3(d, inv);
        if (rc != ORC_OK) return rc;
        w[0] = inv[0];
        w[1] = inv[1];
        w[2] = inv[2];
        return ORC_OK;
    }
    return ORC_ERR_ARG;
}

int orc_cpr_setup(const orc_bcsr *A, int32_t nx, int32_t ny, int32_t nz, int32_t variant, int32_t decouple,
                  orc_apply_fn R, void *Rctx, int32_t coarse_max, int32_t pre, int32_t post, orc_cpr **out,
                  int64_t *bad_cell)
{
    if (bad_cell) *bad_cell = -1;
    if (!A || !out || !R || variant < ORC_CPR_FP || variant > ORC_CPR_FFPF || decouple < ORC_DECOUPLE_NONE ||
        decouple > ORC_DECOUPLE_ABF || A->n != (int64_t)nx * ny * nz)
        return ORC_ERR_ARG;
    const int64_t n = A->n;
    orc_cpr *P = (orc_cpr *)calloc(1, sizeof(orc_cpr));
    if (!P) return ORC_ERR_OOM;
    P->A = A;
    P->n = n;
    P->variant = variant;
    P->decouple = decouple;
    P->R = R;
    P->Rctx = Rctx;
    P->w = (double *)malloc((size_t)(3 * n) * sizeof(double));
    P->r = (double *)malloc((size_t)(3 * n) * sizeof(double));
    P->t = (double *)malloc((size_t)(3 * n) * sizeof(double));
    P->q = (double *)malloc((size_t)n * sizeof(double));
    P->e = (double *)malloc((size_t)n * sizeof(double));
    int64_t *rp = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int64_t *col = (int64_t *)malloc((size_t)(A->nnzb > 0 ? A->nnzb : 1) * sizeof(int64_t));
    double *val = (double *)malloc((size_t)(A->nnzb > 0 ? A->nnzb : 1) * sizeof(double));
    int rc = (P->w && P->r && P->t && P->q && P->e && rp && col && val) ? ORC_OK : ORC_ERR_OOM;
    /* weights from the diagonal blocks */
    for (int64_t c = 0; c < n && rc == ORC_OK; ++c) {
        const double *d = NULL;
        for (int64_t p = A->rowptr[c]; p < A->rowptr[c + 1]; ++p)
            if (A->col[p] == c) d = A->val + 9 * p;
        if (!d) rc = ORC_ERR_ZERO_PIVOT;
        else rc = cell_weights(d, decouple, P->w + 3 * c);
        if (rc != ORC_OK && bad_cell) *bad_cell = c;
    }
    /* A_pp(c, m) = sum_q w_c[q] A_cm[q][0], on the block pattern */
    if (rc == ORC_OK) {
        for (int64_t c = 0; c <= n; ++c) rp[c] = A->rowptr[c];
        for (int64_t c = 0; c < n; ++c)
            for (int64_t p = A->rowptr[c]; p < A->rowptr[c + 1]; ++p) {
                const double *blk = A->val + 9 * p;
                const double *w = P->w + 3 * c;
                col[p] = A->col[p];
                val[p] = w[0] * blk[0] + w[1] * blk[3] + w[2] * blk[6];
            }
        rc = orc_csr_from_arrays(n, rp, col, val, &P->App);
    }
    if (rc == ORC_OK) rc = orc_mg_setup(P->App, nx, ny, nz, coarse_max, pre, post, &P->mg);
    free(rp);
    free(col);
    free(val);
    if (rc != ORC_OK) {
        orc_cpr_free(P);
        return rc;
    }
    *out = P;
    return ORC_OK;
}

/* r = f - A x */
static void residual(const orc_cpr *P, const double *f, const double *x, double *r)
{
    orc_spmv(P->A, x, r);
    for (int64_t i = 0; i < 3 * P->n; ++i) r[i] = f[i] - r[i];
}

/* x += Pi_p M_g^-1 (Pi_r of the decoupled r) */
static int pressure_step(orc_cpr *P, const double *r, double *x)
{
    for (int64_t c = 0; c < P->n; ++c) {
        const double *w = P->w + 3 * c;
        P->q[c] = w[0] * r[3 * c] + w[1] * r[3 * c + 1] + w[2] * r[3 * c + 2];
    }
    const int rc = orc_mg_apply(P->mg, P->q, P->e);
    if (rc != ORC_OK) return rc;
    for (int64_t c = 0; c < P->n; ++c) x[3 * c] += P->e[c];
    return ORC_OK;
}

/* x += R^-1 r */
static int smoother_step(orc_cpr *P, const double *r, double *x)
{
    const int rc = P->R(P->Rctx, r, P->t);
    if (rc != ORC_OK) return rc;
    for (int64_t i = 0; i < 3 * P->n; ++i) x[i] += P->t[i];
    return ORC_OK;
}

int orc_cpr_apply(void *ctx, const double *f, double *x)
{
    orc_cpr *P = (orc_cpr *)ctx;
    if (!P || !f || !x) return ORC_ERR_ARG;
    const int64_t N = 3 * P->n;
    int rc;
    for (int64_t i = 0; i < N; ++i) x[i] = 0.0;
    switch (P->variant) {
    case ORC_CPR_FP:          /* x = R f; r = f - A x; pressure */
        if ((rc = smoother_step(P, f, x)) != ORC_OK) return rc;
        residual(P, f, x, P->r);
        if ((rc = pressure_step(P, P->r, x)) != ORC_OK) return rc;
        break;
    case ORC_CPR_PF:          /* pressure of f; r = f - A x; x += R r */
        if ((rc = pressure_step(P, f, x)) != ORC_OK) return rc;
        residual(P, f, x, P->r);
        if ((rc = smoother_step(P, P->r, x)) != ORC_OK) return rc;
        break;
    case ORC_CPR_FPF:         /* x = R f; pressure; x += R r */
        if ((rc = smoother_step(P, f, x)) != ORC_OK) return rc;
        residual(P, f, x, P->r);
        if ((rc = pressure_step(P, P->r, x)) != ORC_OK) return rc;
        residual(P, f, x, P->r);
        if ((rc = smoother_step(P, P->r, x)) != ORC_OK) return rc;
        break;
    case ORC_CPR_FFPF:        /* x = R f; x += R r; pressure; x += R r */
        if ((rc = smoother_step(P, f, x)) != ORC_OK) return rc;
        residual(P, f, x, P->r);
        if ((rc = smoother_step(P, P->r, x)) != ORC_OK) return rc;
        residual(P, f, x, P->r);
        if ((rc = pressure_step(P, P->r, x)) != ORC_OK) return rc;
        residual(P, f, x, P->r);
        if ((rc = smoother_step(P, P->r, x)) != ORC_OK) return rc;
        break;
    default:
        return ORC_ERR_ARG;
    }
    for (int64_t i = 0; i < N; ++i)
        if (!isfinite(x[i])) return ORC_ERR_NAN;
    return ORC_OK;
}

void orc_cpr_weights(const orc_cpr *P, double *w) { memcpy(w, P->w, (size_t)(3 * P->n) * sizeof(double)); }
const orc_csr *orc_cpr_pressure_matrix(const orc_cpr *P) { return P->App; }
const orc_mg *orc_cpr_mg(const orc_cpr *P) { return P->mg; }
