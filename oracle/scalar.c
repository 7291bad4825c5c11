/*
 * CPU ORACLE -- test infrastructure only.  The scalar (one unknown per cell)
 * counterparts of the block routines in oracle.c, for the paper's Poisson
 * Equation example: GMRES(30) with RAS, overlap one, ILU(0) on every
 * subdomain.  Plain serial FP64, sharing no code with the GPU library.
 *
 *  - storage: CSR with ascending columns, built from 7-point coefficients
 *    (slots -z,-y,-x,D,+x,+y,+z), absent neighbours omitted;
 *  - ILU(0): the textbook IKJ form (Saad, Iterative Methods for Sparse
 *    Linear Systems, 2nd ed., sec. 10.3) on the pattern of A;
 *  - RAS: restricted additive Schwarz (Cai & Sarkis 1999, the paper's [DDM]
 *    citation): px x py x pz boxes (the first n mod p boxes one cell longer),
 *    Omega_s = cells within matrix-graph distance <= overlap of the box, the
 *    local matrix is A restricted to Omega_s in ascending global order,
 *    factored by ILU(0), and each cell is written back only by its owner;
 *  - GMRES(m) and BiCGSTAB: the operator versions of oracle.c's drivers.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

struct orc_csr {
    int64_t n, nnz;
    int64_t *rowptr, *col;
    double *val;
};

static orc_csr *csr_alloc(int64_t n, int64_t nnz)
{
    orc_csr *A = (orc_csr *)calloc(1, sizeof(orc_csr));
    if (!A) return NULL;
    A->n = n;
    A->nnz = nnz;
    A->rowptr = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    A->col = (int64_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
    A->val = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    if (!A->rowptr || !A->col || !A->val) {
        orc_csr_free(A);
        return NULL;
    }
    return A;
}

void orc_csr_free(orc_csr *A)
{
    if (!A) return;
    free(A->rowptr);
    free(A->col);
    free(A->val);
    free(A);
}

int64_t orc_csr_nnz(const orc_csr *A) { return A->nnz; }

void orc_csr_export(const orc_csr *A, int64_t *rowptr, int64_t *col, double *val)
{
    memcpy(rowptr, A->rowptr, (size_t)(A->n + 1) * sizeof(int64_t));
    memcpy(col, A->col, (size_t)A->nnz * sizeof(int64_t));
    memcpy(val, A->val, (size_t)A->nnz * sizeof(double));
}

int orc_csr_from_stencil(int32_t nx, int32_t ny, int32_t nz, const double *coef, orc_csr **out)
{
    if (nx < 1 || ny < 1 || nz < 1 || !coef || !out) return ORC_ERR_ARG;
    static const int OFF[7][3] = {{0, 0, -1}, {0, -1, 0}, {-1, 0, 0}, {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    const int64_t n = (int64_t)nx * ny * nz;
    int64_t nnz = 0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i)
                for (int s = 0; s < 7; ++s) {
                    const int64_t ii = i + OFF[s][0], jj = j + OFF[s][1], kk = k + OFF[s][2];
                    const int inside = ii >= 0 && ii < nx && jj >= 0 && jj < ny && kk >= 0 && kk < nz;
                    const double v = coef[7 * ((k * ny + j) * nx + i) + s];
                    if (!isfinite(v)) return ORC_ERR_NAN;
                    if (!inside && v != 0.0) return ORC_ERR_PATTERN;
                    if (inside) ++nnz;
                }
    orc_csr *A = csr_alloc(n, nnz);
    if (!A) return ORC_ERR_OOM;
    int64_t p = 0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t c = (k * ny + j) * nx + i;
                A->rowptr[c] = p;
                for (int s = 0; s < 7; ++s) {   /* slot order is ascending column order */
                    const int64_t ii = i + OFF[s][0], jj = j + OFF[s][1], kk = k + OFF[s][2];
                    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
                    A->col[p] = (kk * ny + jj) * nx + ii;
                    A->val[p] = coef[7 * c + s];
                    ++p;
                }
            }
    A->rowptr[n] = p;
    *out = A;
    return ORC_OK;
}

int orc_csr_from_arrays(int64_t n, const int64_t *rowptr, const int64_t *col, const double *val, orc_csr **out)
{
    if (n < 0 || !rowptr || !out) return ORC_ERR_ARG;
    const int64_t nnz = rowptr[n];
    if (nnz < 0 || (nnz > 0 && (!col || !val))) return ORC_ERR_ARG;
    for (int64_t i = 0; i < n; ++i) {
        if (rowptr[i + 1] < rowptr[i]) return ORC_ERR_ARG;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (col[p] < 0 || col[p] >= n || (p > rowptr[i] && col[p] <= col[p - 1])) return ORC_ERR_ARG;
            if (!isfinite(val[p])) return ORC_ERR_NAN;
        }
    }
    orc_csr *A = csr_alloc(n, nnz);
    if (!A) return ORC_ERR_OOM;
    memcpy(A->rowptr, rowptr, (size_t)(n + 1) * sizeof(int64_t));
    if (nnz > 0) {
        memcpy(A->col, col, (size_t)nnz * sizeof(int64_t));
        memcpy(A->val, val, (size_t)nnz * sizeof(double));
    }
    *out = A;
    return ORC_OK;
}

void orc_csr_view(const orc_csr *A, int64_t *n, const int64_t **rowptr, const int64_t **col, const double **val)
{
    *n = A->n;
    *rowptr = A->rowptr;
    *col = A->col;
    *val = A->val;
}

void orc_csr_spmv(const orc_csr *A, const double *x, double *y)
{
    for (int64_t i = 0; i < A->n; ++i) {
        double s = 0.0;
        for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) s += A->val[p] * x[A->col[p]];
        y[i] = s;
    }
}

static void csr_mv(const void *ctx, const double *x, double *y) { orc_csr_spmv((const orc_csr *)ctx, x, y); }

/* ---- ILU(0) ---- */
struct orc_silu {
    orc_csr *LU;      /* strict lower part: L (unit diagonal implied); upper incl. diagonal: U */
    int64_t *diag;
};

void orc_silu_free(orc_silu *F)
{
    if (!F) return;
    orc_csr_free(F->LU);
    free(F->diag);
    free(F);
}

int orc_csr_ilu0(const orc_csr *A, orc_silu **out, int64_t *bad_row)
{
    if (!A || !out) return ORC_ERR_ARG;
    if (bad_row) *bad_row = -1;
    const int64_t n = A->n;
    orc_silu *F = (orc_silu *)calloc(1, sizeof(orc_silu));
    if (!F) return ORC_ERR_OOM;
    F->LU = csr_alloc(n, A->nnz);
    F->diag = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *where = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!F->LU || !F->diag || !where) {
        free(where);
        orc_silu_free(F);
        return ORC_ERR_OOM;
    }
    orc_csr *M = F->LU;
    memcpy(M->rowptr, A->rowptr, (size_t)(n + 1) * sizeof(int64_t));
    memcpy(M->col, A->col, (size_t)A->nnz * sizeof(int64_t));
    memcpy(M->val, A->val, (size_t)A->nnz * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        F->diag[i] = -1;
        for (int64_t p = M->rowptr[i]; p < M->rowptr[i + 1]; ++p)
            if (M->col[p] == i) F->diag[i] = p;
        where[i] = -1;
    }
    int rc = ORC_OK;
    for (int64_t i = 0; i < n && rc == ORC_OK; ++i) {
        if (F->diag[i] < 0) { rc = ORC_ERR_ZERO_PIVOT; if (bad_row) *bad_row = i; break; }
        for (int64_t p = M->rowptr[i]; p < M->rowptr[i + 1]; ++p) where[M->col[p]] = p;
        /* for each k < i in row i, ascending: a_ik <- a_ik / u_kk, then
         * a_ij <- a_ij - a_ik u_kj for j > k with (i,j) in the pattern */
        for (int64_t p = M->rowptr[i]; p < M->rowptr[i + 1]; ++p) {
            const int64_t k = M->col[p];
            if (k >= i) break;
            M->val[p] /= M->val[F->diag[k]];
            for (int64_t q = M->rowptr[k]; q < M->rowptr[k + 1]; ++q) {
                const int64_t j = M->col[q];
                if (j <= k || where[j] < 0) continue;
                M->val[where[j]] -= M->val[p] * M->val[q];
            }
        }
        const double piv = M->val[F->diag[i]];
        if (!(fabs(piv) > 1e-300) || !isfinite(piv)) { rc = ORC_ERR_ZERO_PIVOT; if (bad_row) *bad_row = i; }
        for (int64_t p = M->rowptr[i]; p < M->rowptr[i + 1]; ++p) where[M->col[p]] = -1;
    }
    free(where);
    if (rc != ORC_OK) {
        orc_silu_free(F);
        return rc;
    }
    *out = F;
    return ORC_OK;
}

const orc_csr *orc_silu_factors(const orc_silu *F) { return F->LU; }

/* z = U^{-1} L^{-1} r: forward y_i = r_i - sum_{k<i} l_ik y_k, backward
 * z_i = (y_i - sum_{j>i} u_ij z_j) / u_ii */
int orc_silu_apply(void *ctx, const double *r, double *z)
{
    const orc_silu *F = (const orc_silu *)ctx;
    const orc_csr *M = F->LU;
    const int64_t n = M->n;
    double *y = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!y) return ORC_ERR_OOM;
    for (int64_t i = 0; i < n; ++i) {
        double s = r[i];
        for (int64_t p = M->rowptr[i]; p < F->diag[i]; ++p) s -= M->val[p] * y[M->col[p]];
        y[i] = s;
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int64_t p = F->diag[i] + 1; p < M->rowptr[i + 1]; ++p) s -= M->val[p] * z[M->col[p]];
        z[i] = s / M->val[F->diag[i]];
    }
    free(y);
    return ORC_OK;
}

/* ---- RAS ---- */
struct orc_sras {
    int64_t n, nsub;
    int64_t *owner;
    int64_t *sub_ptr, *sub_cells;
    orc_silu **local;
};

void orc_sras_free(orc_sras *R)
{
    if (!R) return;
    if (R->local)
        for (int64_t s = 0; s < R->nsub; ++s) orc_silu_free(R->local[s]);
    free(R->local);
    free(R->owner);
    free(R->sub_ptr);
    free(R->sub_cells);
    free(R);
}

/* first index of box b when [0, len) is split into p parts, the first len % p one longer */
static int64_t box_start(int64_t b, int64_t len, int64_t p)
{
    const int64_t base = len / p, rem = len % p;
    return b * base + (b < rem ? b : rem);
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

int orc_sras_setup(const orc_csr *A, int32_t nx, int32_t ny, int32_t nz, int32_t px, int32_t py, int32_t pz,
                   int32_t overlap, orc_sras **out, int64_t *bad_row)
{
    if (!A || !out || px < 1 || py < 1 || pz < 1 || overlap < 0 || px > nx || py > ny || pz > nz) return ORC_ERR_ARG;
    const int64_t n = A->n;
    if (n != (int64_t)nx * ny * nz) return ORC_ERR_ARG;
    if (bad_row) *bad_row = -1;
    orc_sras *R = (orc_sras *)calloc(1, sizeof(orc_sras));
    if (!R) return ORC_ERR_OOM;
    R->n = n;
    R->nsub = (int64_t)px * py * pz;
    R->owner = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    R->sub_ptr = (int64_t *)calloc((size_t)(R->nsub + 1), sizeof(int64_t));
    R->local = (orc_silu **)calloc((size_t)R->nsub, sizeof(orc_silu *));
    int64_t *dist = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *g2l = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t cap = 1024, total = 0;
    int64_t *all = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    int rc = (R->owner && R->sub_ptr && R->local && dist && g2l && all) ? ORC_OK : ORC_ERR_OOM;
    if (rc == ORC_OK) {
        for (int64_t c = 0; c < n; ++c) { dist[c] = -1; g2l[c] = -1; }
    }
    /* owners and Omega_s (breadth-first search over the pattern of A from the box) */
    for (int64_t s = 0; s < R->nsub && rc == ORC_OK; ++s) {
        const int64_t sx = s % px, sy = (s / px) % py, sz = s / ((int64_t)px * py);
        const int64_t x0 = box_start(sx, nx, px), x1 = box_start(sx + 1, nx, px);
        const int64_t y0 = box_start(sy, ny, py), y1 = box_start(sy + 1, ny, py);
        const int64_t z0 = box_start(sz, nz, pz), z1 = box_start(sz + 1, nz, pz);
        const int64_t head0 = total;
        for (int64_t k = z0; k < z1; ++k)
            for (int64_t j = y0; j < y1; ++j)
                for (int64_t i = x0; i < x1; ++i) {
                    const int64_t c = (k * ny + j) * nx + i;
                    R->owner[c] = s;
                    if (total == cap) {
                        cap *= 2;
                        int64_t *t = (int64_t *)realloc(all, (size_t)cap * sizeof(int64_t));
                        if (!t) { rc = ORC_ERR_OOM; break; }
                        all = t;
                    }
                    all[total++] = c;
                    dist[c] = 0;
                }
        for (int64_t h = head0; h < total && rc == ORC_OK; ++h) {
            const int64_t c = all[h];
            if (dist[c] >= overlap) continue;
            for (int64_t p = A->rowptr[c]; p < A->rowptr[c + 1]; ++p) {
                const int64_t nb = A->col[p];
                if (dist[nb] >= 0) continue;
                dist[nb] = dist[c] + 1;
                if (total == cap) {
                    cap *= 2;
                    int64_t *t = (int64_t *)realloc(all, (size_t)cap * sizeof(int64_t));
                    if (!t) { rc = ORC_ERR_OOM; break; }
                    all = t;
                }
                all[total++] = nb;
            }
        }
        for (int64_t h = head0; h < total; ++h) dist[all[h]] = -1;
        qsort(all + head0, (size_t)(total - head0), sizeof(int64_t), cmp_i64);
        R->sub_ptr[s + 1] = total;
    }
    R->sub_cells = all;
    /* local matrices: A restricted to Omega_s (couplings leaving it dropped), ILU(0) each */
    for (int64_t s = 0; s < R->nsub && rc == ORC_OK; ++s) {
        const int64_t *cs = all + R->sub_ptr[s];
        const int64_t m = R->sub_ptr[s + 1] - R->sub_ptr[s];
        for (int64_t q = 0; q < m; ++q) g2l[cs[q]] = q;
        int64_t nnz = 0;
        for (int64_t q = 0; q < m; ++q)
            for (int64_t p = A->rowptr[cs[q]]; p < A->rowptr[cs[q] + 1]; ++p)
                if (g2l[A->col[p]] >= 0) ++nnz;
        orc_csr *As = csr_alloc(m, nnz);
        if (!As) { rc = ORC_ERR_OOM; break; }
        int64_t pos = 0;
        for (int64_t q = 0; q < m; ++q) {
            As->rowptr[q] = pos;
            for (int64_t p = A->rowptr[cs[q]]; p < A->rowptr[cs[q] + 1]; ++p) {
                const int64_t lc = g2l[A->col[p]];
                if (lc < 0) continue;
                As->col[pos] = lc;
                As->val[pos] = A->val[p];
                ++pos;
            }
        }
        As->rowptr[m] = pos;
        int64_t bad = -1;
        rc = orc_csr_ilu0(As, &R->local[s], &bad);
        if (rc != ORC_OK && bad_row) *bad_row = bad >= 0 ? cs[bad] : -1;
        orc_csr_free(As);
        for (int64_t q = 0; q < m; ++q) g2l[cs[q]] = -1;
    }
    free(dist);
    free(g2l);
    if (rc != ORC_OK) {
        orc_sras_free(R);
        return rc;
    }
    *out = R;
    return ORC_OK;
}

int64_t orc_sras_nsub(const orc_sras *R) { return R->nsub; }
int64_t orc_sras_sub_size(const orc_sras *R, int64_t s) { return R->sub_ptr[s + 1] - R->sub_ptr[s]; }
void orc_sras_sub_cells(const orc_sras *R, int64_t s, int64_t *cells)
{
    memcpy(cells, R->sub_cells + R->sub_ptr[s], (size_t)orc_sras_sub_size(R, s) * sizeof(int64_t));
}

int orc_sras_apply(void *ctx, const double *r, double *z)
{
    const orc_sras *R = (const orc_sras *)ctx;
    int64_t maxm = 1;
    for (int64_t s = 0; s < R->nsub; ++s)
        if (orc_sras_sub_size(R, s) > maxm) maxm = orc_sras_sub_size(R, s);
    double *rl = (double *)malloc((size_t)maxm * sizeof(double));
    double *zl = (double *)malloc((size_t)maxm * sizeof(double));
    if (!rl || !zl) { free(rl); free(zl); return ORC_ERR_OOM; }
    for (int64_t s = 0; s < R->nsub; ++s) {
        const int64_t *cs = R->sub_cells + R->sub_ptr[s];
        const int64_t m = orc_sras_sub_size(R, s);
        for (int64_t q = 0; q < m; ++q) rl[q] = r[cs[q]];
        orc_silu_apply(R->local[s], rl, zl);
        for (int64_t q = 0; q < m; ++q)
            if (R->owner[cs[q]] == s) z[cs[q]] = zl[q];
    }
    free(rl);
    free(zl);
    return ORC_OK;
}

/* ---- Krylov methods on the scalar operator ---- */
int orc_csr_gmres(const orc_csr *A, orc_apply_fn pc, void *pc_ctx, const double *b, double *x, int32_t m,
                  double tol, int64_t maxit, orc_stats *st, double *hist)
{
    if (!A) return ORC_ERR_ARG;
    return orc_gmres_op(A->n, csr_mv, A, pc, pc_ctx, b, x, m, tol, maxit, st, hist);
}

int orc_csr_bicgstab(const orc_csr *A, orc_apply_fn pc, void *pc_ctx, const double *b, double *x, double tol,
                     int64_t maxit, orc_stats *st, double *hist)
{
    if (!A) return ORC_ERR_ARG;
    return orc_bicgstab_op(A->n, csr_mv, A, pc, pc_ctx, b, x, tol, maxit, st, hist);
}
