/*
 * CPU ORACLE -- test infrastructure only.  The pressure solve of the CPR-type
 * preconditioners (the paper's CPR-like Preconditioners subsection writes it
 * M_g(A_pp)^-1 and uses algebraic multigrid from a library there): one
 * V-cycle of an aggregation multigrid on the structured grid.  Plain serial
 * FP64, sharing no code with the GPU library.
 *
 *  - levels: level 0 is the given matrix on an nx x ny x nz grid, row
 *    r = i + nx (j + ny k).  Level l+1 aggregates the cells of level l in
 *    2 x 2 x 2 boxes: cell (i, j, k) belongs to aggregate (i/2, j/2, k/2), so
 *    an axis of one cell stays one cell and an odd axis ends in aggregates one
 *    cell thick.  Coarsening stops at the first level with at most coarse_max
 *    cells (or one cell);
 *  - coarse operators: Galerkin, A_{l+1} = P^T A_l P with P the 0/1 matrix
 *    of cell-to-aggregate membership, i.e. A_{l+1}(I, J) is the sum of
 *    A_l(i, j) over i in I and j in J (aggregation without smoothing of the
 *    prolongation, as in Braess 1995);
 *  - smoothing: Gauss-Seidel over the cells of one colour, then the other,
 *    colour (i + j + k) mod 2, red = 0.  Pre-smoothing: `pre` sweeps of red
 *    then black; post-smoothing: `post` sweeps of black then red, so that for
 *    a symmetric matrix the cycle is a symmetric operator;
 *  - coarsest level: Gaussian elimination with partial pivoting, factored
 *    once at setup;
 *  - cycle on level l for right-hand side b: x = 0, pre-smooth, r = b - A x,
 *    b_{l+1} = P^T r, x_{l+1} = cycle(l + 1), x += P x_{l+1}, post-smooth.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MG_MAX_LEVELS 40
#define MG_ROW_CAP 64   /* distinct coarse columns per coarse row the builder accepts */

typedef struct mg_level {
    int32_t nx, ny, nz;
    int64_t n;
    orc_csr *A;
    double *b, *x, *r;
} mg_level;

struct orc_mg {
    int32_t nlev, pre, post;
    mg_level lev[MG_MAX_LEVELS];
    double *lu;       /* coarsest level: n x n LU factors, row-major */
    int64_t *piv;     /* row interchanges */
};

static int64_t ceil_half(int32_t v) { return v > 1 ? (v + 1) / 2 : 1; }

static int64_t aggregate_of(const mg_level *f, int64_t row, int32_t cnx, int32_t cny)
{
    const int64_t i = row % f->nx, j = (row / f->nx) % f->ny, k = row / ((int64_t)f->nx * f->ny);
    const int64_t ci = f->nx > 1 ? i / 2 : 0, cj = f->ny > 1 ? j / 2 : 0, ck = f->nz > 1 ? k / 2 : 0;
    return (ck * cny + cj) * cnx + ci;
}

/* A_c = P^T A P by summing every fine entry into its aggregate pair, in
 * ascending fine row, then ascending fine column */
static int galerkin(const mg_level *f, mg_level *c)
{
    int64_t n;
    const int64_t *rp, *col;
    const double *val;
    orc_csr_view(f->A, &n, &rp, &col, &val);
    const int64_t nc = c->n;
    int64_t *ccnt = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
    int64_t *ccol = (int64_t *)malloc((size_t)nc * MG_ROW_CAP * sizeof(int64_t));
    double *cval = (double *)malloc((size_t)nc * MG_ROW_CAP * sizeof(double));
    if (!ccnt || !ccol || !cval) {
        free(ccnt); free(ccol); free(cval);
        return ORC_ERR_OOM;
    }
    int rc = ORC_OK;
    for (int64_t i = 0; i < n && rc == ORC_OK; ++i) {
        const int64_t I = aggregate_of(f, i, c->nx, c->ny);
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int64_t J = aggregate_of(f, col[p], c->nx, c->ny);
            int64_t q = 0;
            while (q < ccnt[I] && ccol[I * MG_ROW_CAP + q] != J) ++q;
            if (q == ccnt[I]) {
                if (q == MG_ROW_CAP) { rc = ORC_ERR_ARG; break; }
                ccol[I * MG_ROW_CAP + q] = J;
                cval[I * MG_ROW_CAP + q] = 0.0;
                ++ccnt[I];
            }
            cval[I * MG_ROW_CAP + q] += val[p];
        }
    }
    if (rc == ORC_OK) {
        /* columns ascending within each coarse row (insertion sort) */
        int64_t *crp = (int64_t *)malloc((size_t)(nc + 1) * sizeof(int64_t));
        int64_t *cc = (int64_t *)malloc((size_t)(nc * MG_ROW_CAP + 1) * sizeof(int64_t));
        double *cv = (double *)malloc((size_t)(nc * MG_ROW_CAP + 1) * sizeof(double));
        if (!crp || !cc || !cv) rc = ORC_ERR_OOM;
        int64_t pos = 0;
        for (int64_t I = 0; I < nc && rc == ORC_OK; ++I) {
            crp[I] = pos;
            int64_t *rc_ = ccol + I * MG_ROW_CAP;
            double *rv = cval + I * MG_ROW_CAP;
            for (int64_t a = 1; a < ccnt[I]; ++a) {
                const int64_t kc = rc_[a];
                const double kv = rv[a];
                int64_t b = a - 1;
                while (b >= 0 && rc_[b] > kc) {
                    rc_[b + 1] = rc_[b];
                    rv[b + 1] = rv[b];
                    --b;
                }
                rc_[b + 1] = kc;
                rv[b + 1] = kv;
            }
            for (int64_t a = 0; a < ccnt[I]; ++a) {
                cc[pos] = rc_[a];
                cv[pos] = rv[a];
                ++pos;
            }
        }
        if (rc == ORC_OK) {
            crp[nc] = pos;
            rc = orc_csr_from_arrays(nc, crp, cc, cv, &c->A);
        }
        free(crp); free(cc); free(cv);
    }
    free(ccnt); free(ccol); free(cval);
    return rc;
}

/* Gauss-Seidel over the rows of one colour, in ascending order */
static int gs_colour(const mg_level *L, const double *b, double *x, int colour)
{
    int64_t n;
    const int64_t *rp, *col;
    const double *val;
    orc_csr_view(L->A, &n, &rp, &col, &val);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t ci = i % L->nx, cj = (i / L->nx) % L->ny, ck = i / ((int64_t)L->nx * L->ny);
        if ((int)((ci + cj + ck) & 1) != colour) continue;
        double s = b[i], d = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (col[p] == i) d = val[p];
            else s -= val[p] * x[col[p]];
        }
        if (d == 0.0) return ORC_ERR_ZERO_PIVOT;
        x[i] = s / d;
    }
    return ORC_OK;
}

static int dense_factor(orc_mg *M)
{
    const mg_level *L = &M->lev[M->nlev - 1];
    const int64_t n = L->n;
    M->lu = (double *)calloc((size_t)(n * n), sizeof(double));
    M->piv = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!M->lu || !M->piv) return ORC_ERR_OOM;
    int64_t nn;
    const int64_t *rp, *col;
    const double *val;
    orc_csr_view(L->A, &nn, &rp, &col, &val);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) M->lu[i * n + col[p]] = val[p];
    double *a = M->lu;
    for (int64_t c = 0; c < n; ++c) {
        int64_t pr = c;
        for (int64_t r = c + 1; r < n; ++r)
            if (fabs(a[r * n + c]) > fabs(a[pr * n + c])) pr = r;
        if (!(fabs(a[pr * n + c]) > 1e-300)) return ORC_ERR_ZERO_PIVOT;
        M->piv[c] = pr;
        if (pr != c)
            for (int64_t q = 0; q < n; ++q) {
                const double t = a[c * n + q];
                a[c * n + q] = a[pr * n + q];
                a[pr * n + q] = t;
            }
        for (int64_t r = c + 1; r < n; ++r) {
            const double f = a[r * n + c] / a[c * n + c];
            a[r * n + c] = f;
            for (int64_t q = c + 1; q < n; ++q) a[r * n + q] -= f * a[c * n + q];
        }
    }
    return ORC_OK;
}

static void dense_solve(const orc_mg *M, const double *b, double *x)
{
    const int64_t n = M->lev[M->nlev - 1].n;
    const double *a = M->lu;
    memcpy(x, b, (size_t)n * sizeof(double));
    for (int64_t c = 0; c < n; ++c)
        if (M->piv[c] != c) {
            const double t = x[c];
            x[c] = x[M->piv[c]];
            x[M->piv[c]] = t;
        }
    for (int64_t r = 0; r < n; ++r)
        for (int64_t q = 0; q < r; ++q) x[r] -= a[r * n + q] * x[q];
    for (int64_t r = n - 1; r >= 0; --r) {
        for (int64_t q = r + 1; q < n; ++q) x[r] -= a[r * n + q] * x[q];
        x[r] /= a[r * n + r];
    }
}

void orc_mg_free(orc_mg *M)
{
    if (!M) return;
    for (int l = 0; l < M->nlev; ++l) {
        if (l > 0) orc_csr_free(M->lev[l].A);
        free(M->lev[l].b);
        free(M->lev[l].x);
        free(M->lev[l].r);
    }
    free(M->lu);
    free(M->piv);
    free(M);
}

int orc_mg_setup(const orc_csr *A, int32_t nx, int32_t ny, int32_t nz, int32_t coarse_max, int32_t pre,
                 int32_t post, orc_mg **out)
{
    if (!A || !out || nx < 1 || ny < 1 || nz < 1 || coarse_max < 1 || pre < 0 || post < 0) return ORC_ERR_ARG;
    int64_t n;
    const int64_t *rp, *col;
    const double *val;
    orc_csr_view(A, &n, &rp, &col, &val);
    if (n != (int64_t)nx * ny * nz) return ORC_ERR_ARG;
    orc_mg *M = (orc_mg *)calloc(1, sizeof(orc_mg));
    if (!M) return ORC_ERR_OOM;
    M->pre = pre;
    M->post = post;
    M->lev[0].nx = nx;
    M->lev[0].ny = ny;
    M->lev[0].nz = nz;
    M->lev[0].n = n;
    M->lev[0].A = (orc_csr *)A;   /* not owned */
    M->nlev = 1;
    int rc = ORC_OK;
    while (rc == ORC_OK) {
        mg_level *f = &M->lev[M->nlev - 1];
        f->b = (double *)calloc((size_t)f->n, sizeof(double));
        f->x = (double *)calloc((size_t)f->n, sizeof(double));
        f->r = (double *)calloc((size_t)f->n, sizeof(double));
        if (!f->b || !f->x || !f->r) { rc = ORC_ERR_OOM; break; }
        if (f->n <= coarse_max || f->n == 1) break;
        if (M->nlev == MG_MAX_LEVELS) { rc = ORC_ERR_ARG; break; }
        mg_level *c = &M->lev[M->nlev];
        c->nx = (int32_t)ceil_half(f->nx);
        c->ny = (int32_t)ceil_half(f->ny);
        c->nz = (int32_t)ceil_half(f->nz);
        c->n = (int64_t)c->nx * c->ny * c->nz;
        M->nlev++;
        rc = galerkin(f, c);
    }
    if (rc == ORC_OK) rc = dense_factor(M);
    if (rc != ORC_OK) {
        orc_mg_free(M);
        return rc;
    }
    *out = M;
    return ORC_OK;
}

static int cycle(orc_mg *M, int l, const double *b, double *x)
{
    mg_level *L = &M->lev[l];
    if (l == M->nlev - 1) {
        dense_solve(M, b, x);
        return ORC_OK;
    }
    int rc;
    for (int64_t i = 0; i < L->n; ++i) x[i] = 0.0;
    for (int s = 0; s < M->pre; ++s) {
        if ((rc = gs_colour(L, b, x, 0)) != ORC_OK) return rc;
        if ((rc = gs_colour(L, b, x, 1)) != ORC_OK) return rc;
    }
    orc_csr_spmv(L->A, x, L->r);
    for (int64_t i = 0; i < L->n; ++i) L->r[i] = b[i] - L->r[i];
    mg_level *C = &M->lev[l + 1];
    for (int64_t I = 0; I < C->n; ++I) C->b[I] = 0.0;
    for (int64_t i = 0; i < L->n; ++i) C->b[aggregate_of(L, i, C->nx, C->ny)] += L->r[i];
    if ((rc = cycle(M, l + 1, C->b, C->x)) != ORC_OK) return rc;
    for (int64_t i = 0; i < L->n; ++i) x[i] += C->x[aggregate_of(L, i, C->nx, C->ny)];
    for (int s = 0; s < M->post; ++s) {
        if ((rc = gs_colour(L, b, x, 1)) != ORC_OK) return rc;
        if ((rc = gs_colour(L, b, x, 0)) != ORC_OK) return rc;
    }
    return ORC_OK;
}

int orc_mg_apply(void *ctx, const double *b, double *x)
{
    orc_mg *M = (orc_mg *)ctx;
    if (!M || !b || !x) return ORC_ERR_ARG;
    int rc = cycle(M, 0, b, x);
    if (rc != ORC_OK) return rc;
    for (int64_t i = 0; i < M->lev[0].n; ++i)
        if (!isfinite(x[i])) return ORC_ERR_NAN;
    return ORC_OK;
}

int32_t orc_mg_levels(const orc_mg *M) { return M->nlev; }

void orc_mg_level_dims(const orc_mg *M, int32_t l, int32_t *dims)
{
    dims[0] = M->lev[l].nx;
    dims[1] = M->lev[l].ny;
    dims[2] = M->lev[l].nz;
}

const orc_csr *orc_mg_level_matrix(const orc_mg *M, int32_t l) { return M->lev[l].A; }

/* one colour sweep, exposed for the pins: level 0 only */
int orc_mg_gs_sweep(const orc_mg *M, const double *b, double *x, int32_t colour)
{
    if (!M || !b || !x || (colour != 0 && colour != 1)) return ORC_ERR_ARG;
    return gs_colour(&M->lev[0], b, x, colour);
}
