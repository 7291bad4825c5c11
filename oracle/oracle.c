/*
 * CPU ORACLE -- test infrastructure only (see oracle.h).  Plain serial FP64.
 * Written for a reader checking it against the paper and the textbook
 * methods it cites, not for speed: no blocking, no fusion, no reordering.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* 3x3 helpers                                                          */
/* ------------------------------------------------------------------ */

/* C = A B */
static void mm3(const double *A, const double *B, double *C)
{
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            double s = 0.0;
            for (int t = 0; t < 3; ++t) s += A[3 * p + t] * B[3 * t + q];
            C[3 * p + q] = s;
        }
}

/* y += A x (3-vectors) */
static void mv3_add(const double *A, const double *x, double *y)
{
    for (int p = 0; p < 3; ++p) {
        double s = 0.0;
        for (int q = 0; q < 3; ++q) s += A[3 * p + q] * x[q];
        y[p] += s;
    }
}

static double norm1_3(const double *a)
{
    double best = 0.0;
    for (int q = 0; q < 3; ++q) {
        double s = fabs(a[q]) + fabs(a[3 + q]) + fabs(a[6 + q]);
        if (s > best) best = s;
    }
    return best;
}

/* Inverse of a 3x3 matrix by LU with partial pivoting, solving for the three
 * unit vectors.  A pivot is treated as zero when |u_pp| <= 1e-300 or when the
 * 1-norm condition estimate exceeds 1e14. */
int orc_inv3(const double *a, double *ainv)
{
    double lu[9];
    int perm[3] = {0, 1, 2};
    memcpy(lu, a, sizeof(lu));
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(lu[3 * r + c]) > fabs(lu[3 * piv + c])) piv = r;
        if (!(fabs(lu[3 * piv + c]) > 1e-300)) return ORC_ERR_ZERO_PIVOT;
        if (piv != c) {
            for (int q = 0; q < 3; ++q) {
                double t = lu[3 * c + q]; lu[3 * c + q] = lu[3 * piv + q]; lu[3 * piv + q] = t;
            }
            int t = perm[c]; perm[c] = perm[piv]; perm[piv] = t;
        }
        for (int r = c + 1; r < 3; ++r) {
            double f = lu[3 * r + c] / lu[3 * c + c];
            lu[3 * r + c] = f;
            for (int q = c + 1; q < 3; ++q) lu[3 * r + q] -= f * lu[3 * c + q];
        }
    }
    for (int col = 0; col < 3; ++col) {
        /* solve L U x = P e_col */
        double y[3];
        for (int r = 0; r < 3; ++r) {
            double v = (perm[r] == col) ? 1.0 : 0.0;
            for (int t = 0; t < r; ++t) v -= lu[3 * r + t] * y[t];
            y[r] = v;
        }
        for (int r = 2; r >= 0; --r) {
            double v = y[r];
            for (int t = r + 1; t < 3; ++t) v -= lu[3 * r + t] * ainv[3 * t + col];
            ainv[3 * r + col] = v / lu[3 * r + r];
        }
    }
    double cond = norm1_3(a) * norm1_3(ainv);
    if (!(cond <= 1e14)) return ORC_ERR_ZERO_PIVOT;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Block CSR storage                                                    */
/* ------------------------------------------------------------------ */

static orc_bcsr *bcsr_alloc(int64_t n, int64_t nnzb)
{
    orc_bcsr *A = (orc_bcsr *)calloc(1, sizeof(orc_bcsr));
    if (!A) return NULL;
    A->n = n;
    A->nnzb = nnzb;
    A->rowptr = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    A->col = (int64_t *)malloc((size_t)(nnzb > 0 ? nnzb : 1) * sizeof(int64_t));
    A->val = (double *)malloc((size_t)(nnzb > 0 ? nnzb : 1) * 9 * sizeof(double));
    if (!A->rowptr || !A->col || !A->val) {
        orc_bcsr_free(A);
        return NULL;
    }
    return A;
}

void orc_bcsr_free(orc_bcsr *A)
{
    if (!A) return;
    free(A->rowptr);
    free(A->col);
    free(A->val);
    free(A);
}

int64_t orc_bcsr_nnzb(const orc_bcsr *A) { return A->nnzb; }

void orc_bcsr_export(const orc_bcsr *A, int64_t *rowptr, int64_t *col, double *val)
{
    memcpy(rowptr, A->rowptr, (size_t)(A->n + 1) * sizeof(int64_t));
    memcpy(col, A->col, (size_t)A->nnzb * sizeof(int64_t));
    memcpy(val, A->val, (size_t)A->nnzb * 9 * sizeof(double));
}

/* Stencil blocks [ncell][7][9] (slots -z,-y,-x,D,+x,+y,+z) -> block CSR in
 * natural cell order C = nx*ny*k + nx*j + i.  A nonzero block in a slot whose
 * neighbour lies outside the grid is a pattern error. */
int orc_bcsr_from_stencil(int32_t nx, int32_t ny, int32_t nz, const double *blocks, orc_bcsr **out)
{
    if (nx < 1 || ny < 1 || nz < 1 || !blocks || !out) return ORC_ERR_ARG;
    const int64_t NX = nx, NY = ny, NZ = nz, n = NX * NY * NZ;
    const int di[7] = {0, 0, -1, 0, 1, 0, 0};
    const int dj[7] = {0, -1, 0, 0, 0, 1, 0};
    const int dk[7] = {-1, 0, 0, 0, 0, 0, 1};
    int64_t nnzb = 0;
    for (int64_t k = 0; k < NZ; ++k)
        for (int64_t j = 0; j < NY; ++j)
            for (int64_t i = 0; i < NX; ++i)
                for (int s = 0; s < 7; ++s) {
                    int64_t ii = i + di[s], jj = j + dj[s], kk = k + dk[s];
                    if (ii >= 0 && ii < NX && jj >= 0 && jj < NY && kk >= 0 && kk < NZ) ++nnzb;
                }
    orc_bcsr *A = bcsr_alloc(n, nnzb);
    if (!A) return ORC_ERR_OOM;
    int64_t pos = 0;
    for (int64_t k = 0; k < NZ; ++k)
        for (int64_t j = 0; j < NY; ++j)
            for (int64_t i = 0; i < NX; ++i) {
                const int64_t C = k * NX * NY + j * NX + i;
                A->rowptr[C] = pos;
                for (int s = 0; s < 7; ++s) {
                    const double *blk = blocks + (C * 7 + s) * 9;
                    int64_t ii = i + di[s], jj = j + dj[s], kk = k + dk[s];
                    if (ii >= 0 && ii < NX && jj >= 0 && jj < NY && kk >= 0 && kk < NZ) {
                        A->col[pos] = kk * NX * NY + jj * NX + ii;
                        memcpy(A->val + 9 * pos, blk, 9 * sizeof(double));
                        ++pos;
                    } else {
                        for (int e = 0; e < 9; ++e)
                            if (blk[e] != 0.0) {
                                orc_bcsr_free(A);
                                return ORC_ERR_PATTERN;
                            }
                    }
                }
            }
    A->rowptr[n] = pos;
    *out = A;
    return ORC_OK;
}

/* General block CSR given by the caller (used by the pins on small graphs). */
int orc_bcsr_from_dense_pattern(int64_t n, const int64_t *rowptr, const int64_t *col, const double *val, orc_bcsr **out)
{
    if (n < 0 || !rowptr || !out) return ORC_ERR_ARG;
    int64_t nnzb = rowptr[n];
    orc_bcsr *A = bcsr_alloc(n, nnzb);
    if (!A) return ORC_ERR_OOM;
    memcpy(A->rowptr, rowptr, (size_t)(n + 1) * sizeof(int64_t));
    memcpy(A->col, col, (size_t)nnzb * sizeof(int64_t));
    memcpy(A->val, val, (size_t)nnzb * 9 * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = A->rowptr[i] + 1; p < A->rowptr[i + 1]; ++p)
            if (A->col[p] <= A->col[p - 1]) {
                orc_bcsr_free(A);
                return ORC_ERR_PATTERN;
            }
    *out = A;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Algebraic operations                                                 */
/* ------------------------------------------------------------------ */

void orc_spmv(const orc_bcsr *A, const double *x, double *y)
{
    for (int64_t i = 0; i < A->n; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
            mv3_add(A->val + 9 * p, x + 3 * A->col[p], acc);
        y[3 * i + 0] = acc[0];
        y[3 * i + 1] = acc[1];
        y[3 * i + 2] = acc[2];
    }
}

double orc_dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

double orc_nrm2(int64_t n, const double *x) { return sqrt(orc_dot(n, x, x)); }

/* ------------------------------------------------------------------ */
/* ILU(0), generic IKJ form on block CSR                                */
/* ------------------------------------------------------------------ */

struct orc_ilu {
    orc_bcsr *LU;     /* strict lower part: L (unit diagonal implied); upper incl. diagonal: U */
    int64_t *diag;    /* position of the diagonal block in each row */
    double  *dinv;    /* 9 per row: inverse of U's diagonal block */
    float   *val32;   /* lazily built FP32 copies */
    float   *dinv32;
};

void orc_ilu_free(orc_ilu *F)
{
    if (!F) return;
    orc_bcsr_free(F->LU);
    free(F->diag);
    free(F->dinv);
    free(F->val32);
    free(F->dinv32);
    free(F);
}

const orc_bcsr *orc_ilu_factors(const orc_ilu *F) { return F->LU; }

/* The numeric IKJ factorisation on the pattern of A (which may hold explicit
 * zero blocks at fill positions): ILU(0) of A when A carries its own pattern,
 * ILU(k) when it carries the level-k pattern. */
static int ilu_numeric(const orc_bcsr *A, orc_ilu **out, int64_t *bad_cell)
{
    if (!A || !out) return ORC_ERR_ARG;
    if (bad_cell) *bad_cell = -1;
    const int64_t n = A->n;
    orc_ilu *F = (orc_ilu *)calloc(1, sizeof(orc_ilu));
    if (!F) return ORC_ERR_OOM;
    F->LU = bcsr_alloc(n, A->nnzb);
    F->diag = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    F->dinv = (double *)malloc((size_t)(n > 0 ? n : 1) * 9 * sizeof(double));
    int64_t *where = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!F->LU || !F->diag || !F->dinv || !where) {
        free(where);
        orc_ilu_free(F);
        return ORC_ERR_OOM;
    }
    memcpy(F->LU->rowptr, A->rowptr, (size_t)(n + 1) * sizeof(int64_t));
    memcpy(F->LU->col, A->col, (size_t)A->nnzb * sizeof(int64_t));
    memcpy(F->LU->val, A->val, (size_t)A->nnzb * 9 * sizeof(double));
    orc_bcsr *M = F->LU;
    for (int64_t i = 0; i < n; ++i) {
        F->diag[i] = -1;
        for (int64_t p = M->rowptr[i]; p < M->rowptr[i + 1]; ++p)
            if (M->col[p] == i) F->diag[i] = p;
        if (F->diag[i] < 0) {
            if (bad_cell) *bad_cell = i;
            free(where);
            orc_ilu_free(F);
            return ORC_ERR_ZERO_PIVOT;
        }
    }
    for (int64_t i = 0; i < n; ++i) where[i] = -1;

    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = M->rowptr[i]; p < M->rowptr[i + 1]; ++p) where[M->col[p]] = p;
        /* for each k < i in row i, ascending: a_ik <- a_ik * U_kk^{-1};
         * then a_ij <- a_ij - a_ik * u_kj for j > k with (i,j) in the pattern */
        for (int64_t p = M->rowptr[i]; p < M->rowptr[i + 1]; ++p) {
            const int64_t k = M->col[p];
            if (k >= i) break;
            double lik[9];
            mm3(M->val + 9 * p, F->dinv + 9 * k, lik);
            memcpy(M->val + 9 * p, lik, sizeof(lik));
            for (int64_t q = M->rowptr[k]; q < M->rowptr[k + 1]; ++q) {
                const int64_t j = M->col[q];
                if (j <= k) continue;
                const int64_t pij = where[j];
                if (pij < 0) continue;
                double prod[9];
                mm3(lik, M->val + 9 * q, prod);
                for (int e = 0; e < 9; ++e) M->val[9 * pij + e] -= prod[e];
            }
        }
        /* row i is final: invert its pivot block */
        int rc = orc_inv3(M->val + 9 * F->diag[i], F->dinv + 9 * i);
        for (int64_t p = M->rowptr[i]; p < M->rowptr[i + 1]; ++p) where[M->col[p]] = -1;
        if (rc != ORC_OK) {
            if (bad_cell) *bad_cell = i;
            free(where);
            orc_ilu_free(F);
            return ORC_ERR_ZERO_PIVOT;
        }
    }
    free(where);
    *out = F;
    return ORC_OK;
}

int orc_ilu0(const orc_bcsr *A, orc_ilu **out, int64_t *bad_cell)
{
    return ilu_numeric(A, out, bad_cell);
}

/* an orc_ilu around finished factors (L strict lower, U upper with its
 * diagonal; the struct takes LU over): the diagonal positions and U_ii^-1 */
int orc_ilu_wrap(orc_bcsr *LU, orc_ilu **out, int64_t *bad_cell)
{
    if (!LU || !out) return ORC_ERR_ARG;
    if (bad_cell) *bad_cell = -1;
    const int64_t n = LU->n;
    orc_ilu *F = (orc_ilu *)calloc(1, sizeof(orc_ilu));
    if (!F) {
        orc_bcsr_free(LU);
        return ORC_ERR_OOM;
    }
    F->LU = LU;
    F->diag = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    F->dinv = (double *)malloc((size_t)(n > 0 ? n : 1) * 9 * sizeof(double));
    if (!F->diag || !F->dinv) {
        orc_ilu_free(F);
        return ORC_ERR_OOM;
    }
    for (int64_t i = 0; i < n; ++i) {
        F->diag[i] = -1;
        for (int64_t p = LU->rowptr[i]; p < LU->rowptr[i + 1]; ++p)
            if (LU->col[p] == i) F->diag[i] = p;
        if (F->diag[i] < 0 || orc_inv3(LU->val + 9 * F->diag[i], F->dinv + 9 * i) != ORC_OK) {
            if (bad_cell) *bad_cell = i;
            orc_ilu_free(F);
            return ORC_ERR_ZERO_PIVOT;
        }
    }
    *out = F;
    return ORC_OK;
}

orc_bcsr *orc_bcsr_new(int64_t n, int64_t nnzb) { return bcsr_alloc(n, nnzb); }

/* Level-of-fill pattern of ILU(k) (Saad, Iterative Methods for Sparse Linear
 * Systems, 2nd ed., sec. 10.3.3): the entries of A have level 0; eliminating
 * with row m < i gives position (i, j), j > m, the level lev(i,m) + lev(m,j)
 * + 1, kept when it is at most k.  Returns the pattern as a block CSR whose
 * new positions hold zero blocks, and the levels (nullable). */
static orc_bcsr *iluk_pattern(const orc_bcsr *A, int32_t k, int64_t **levels_out)
{
    const int64_t n = A->n;
    int64_t *rp = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t cap = A->nnzb + 16, used = 0;
    int64_t *cols = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    int64_t *levs = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    int64_t *lev = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));   /* dense, per row */
    int64_t *row = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));   /* sorted columns of row i */
    if (!rp || !cols || !levs || !lev || !row) {
        free(rp); free(cols); free(levs); free(lev); free(row);
        return NULL;
    }
    for (int64_t j = 0; j < n; ++j) lev[j] = -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t len = 0;
        for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
            row[len++] = A->col[p];
            lev[A->col[p]] = 0;
        }
        /* eliminate with every m < i of the row, ascending; the row grows */
        for (int64_t t = 0; t < len && row[t] < i; ++t) {
            const int64_t m = row[t];
            for (int64_t q = rp[m]; q < rp[m + 1]; ++q) {
                const int64_t j = cols[q];
                if (j <= m) continue;
                const int64_t l = lev[m] + levs[q] + 1;
                if (l > k) continue;
                if (lev[j] < 0) {              /* a new position: insert keeping the row sorted */
                    int64_t u = len;
                    while (u > 0 && row[u - 1] > j) { row[u] = row[u - 1]; --u; }
                    row[u] = j;
                    ++len;
                    lev[j] = l;
                } else if (l < lev[j]) {
                    lev[j] = l;
                }
            }
        }
        if (used + len > cap) {
            while (used + len > cap) cap *= 2;
            int64_t *c2 = (int64_t *)realloc(cols, (size_t)cap * sizeof(int64_t));
            int64_t *l2 = c2 ? (int64_t *)realloc(levs, (size_t)cap * sizeof(int64_t)) : NULL;
            if (!c2 || !l2) {
                free(c2 ? c2 : cols); free(rp); free(levs); free(lev); free(row);
                return NULL;
            }
            cols = c2;
            levs = l2;
        }
        rp[i] = used;
        for (int64_t t = 0; t < len; ++t) {
            cols[used] = row[t];
            levs[used] = lev[row[t]];
            lev[row[t]] = -1;
            ++used;
        }
        rp[i + 1] = used;   /* row i is read by the rows after it */
    }
    orc_bcsr *P = bcsr_alloc(n, used);
    if (P) {
        memcpy(P->rowptr, rp, (size_t)(n + 1) * sizeof(int64_t));
        memcpy(P->col, cols, (size_t)used * sizeof(int64_t));
        memset(P->val, 0, (size_t)used * 9 * sizeof(double));
        for (int64_t i = 0; i < n; ++i) {   /* the entries of A, the rest zero */
            int64_t q = P->rowptr[i];
            for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
                while (P->col[q] != A->col[p]) ++q;
                memcpy(P->val + 9 * q, A->val + 9 * p, 9 * sizeof(double));
            }
        }
    }
    if (levels_out && P) *levels_out = levs;
    else free(levs);
    free(rp); free(cols); free(lev); free(row);
    return P;
}

int orc_iluk(const orc_bcsr *A, int32_t k, orc_ilu **out, int64_t *bad_cell)
{
    if (!A || !out || k < 0) return ORC_ERR_ARG;
    if (k == 0) return ilu_numeric(A, out, bad_cell);
    orc_bcsr *P = iluk_pattern(A, k, NULL);
    if (!P) return ORC_ERR_OOM;
    int rc = ilu_numeric(P, out, bad_cell);
    orc_bcsr_free(P);
    return rc;
}

int orc_iluk_pattern(const orc_bcsr *A, int32_t k, int64_t *rowptr, int64_t *col, int64_t *level, int64_t cap)
{
    if (!A || k < 0) return ORC_ERR_ARG;
    int64_t *levs = NULL;
    orc_bcsr *P = iluk_pattern(A, k, &levs);
    if (!P) return ORC_ERR_OOM;
    const int64_t nnzb = P->nnzb;
    if (rowptr && col && level && nnzb <= cap) {
        memcpy(rowptr, P->rowptr, (size_t)(A->n + 1) * sizeof(int64_t));
        memcpy(col, P->col, (size_t)nnzb * sizeof(int64_t));
        memcpy(level, levs, (size_t)nnzb * sizeof(int64_t));
    }
    orc_bcsr_free(P);
    free(levs);
    return (int)nnzb;
}

/* z = U^{-1} L^{-1} r, row by row: forward y_i = r_i - sum_{k<i} L_ik y_k,
 * backward z_i = U_ii^{-1} (y_i - sum_{j>i} U_ij z_j). */
int orc_ilu_apply(void *ctx, const double *r, double *z)
{
    const orc_ilu *F = (const orc_ilu *)ctx;
    const orc_bcsr *M = F->LU;
    const int64_t n = M->n;
    double *y = (double *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    if (!y) return ORC_ERR_OOM;
    for (int64_t i = 0; i < n; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t p = M->rowptr[i]; p < F->diag[i]; ++p)
            mv3_add(M->val + 9 * p, y + 3 * M->col[p], acc);
        for (int c = 0; c < 3; ++c) y[3 * i + c] = r[3 * i + c] - acc[c];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t p = F->diag[i] + 1; p < M->rowptr[i + 1]; ++p)
            mv3_add(M->val + 9 * p, z + 3 * M->col[p], acc);
        double t[3];
        for (int c = 0; c < 3; ++c) t[c] = y[3 * i + c] - acc[c];
        double zi[3] = {0.0, 0.0, 0.0};
        mv3_add(F->dinv + 9 * i, t, zi);
        for (int c = 0; c < 3; ++c) z[3 * i + c] = zi[c];
    }
    free(y);
    return ORC_OK;
}

/* FP32 form: the FP64 factors (L, U off-diagonal blocks, U_ii^{-1}) rounded
 * once to FP32; both sweeps in FP32 arithmetic on fl32(r); z widened. */
int orc_ilu_apply_f32(void *ctx, const double *r, double *z)
{
    orc_ilu *F = (orc_ilu *)ctx;
    const orc_bcsr *M = F->LU;
    const int64_t n = M->n;
    if (!F->val32) {
        F->val32 = (float *)malloc((size_t)(M->nnzb > 0 ? M->nnzb : 1) * 9 * sizeof(float));
        F->dinv32 = (float *)malloc((size_t)(n > 0 ? n : 1) * 9 * sizeof(float));
        if (!F->val32 || !F->dinv32) return ORC_ERR_OOM;
        for (int64_t e = 0; e < 9 * M->nnzb; ++e) F->val32[e] = (float)M->val[e];
        for (int64_t e = 0; e < 9 * n; ++e) F->dinv32[e] = (float)F->dinv[e];
    }
    float *y = (float *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(float));
    float *zz = (float *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(float));
    if (!y || !zz) { free(y); free(zz); return ORC_ERR_OOM; }
    for (int64_t i = 0; i < n; ++i) {
        float v[3] = {(float)r[3 * i], (float)r[3 * i + 1], (float)r[3 * i + 2]};
        for (int64_t p = M->rowptr[i]; p < F->diag[i]; ++p) {
            const float *Lb = F->val32 + 9 * p;
            const float *yk = y + 3 * M->col[p];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) v[a] -= Lb[3 * a + b] * yk[b];
        }
        for (int c = 0; c < 3; ++c) y[3 * i + c] = v[c];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        float v[3] = {y[3 * i], y[3 * i + 1], y[3 * i + 2]};
        for (int64_t p = F->diag[i] + 1; p < M->rowptr[i + 1]; ++p) {
            const float *Ub = F->val32 + 9 * p;
            const float *zj = zz + 3 * M->col[p];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) v[a] -= Ub[3 * a + b] * zj[b];
        }
        const float *Di = F->dinv32 + 9 * i;
        for (int a = 0; a < 3; ++a) {
            float s = 0.0f;
            for (int b = 0; b < 3; ++b) s += Di[3 * a + b] * v[b];
            zz[3 * i + a] = s;
        }
    }
    for (int64_t e = 0; e < 3 * n; ++e) z[e] = (double)zz[e];
    free(y);
    free(zz);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Restricted additive Schwarz (Cai & Sarkis 1999)                      */
/* ------------------------------------------------------------------ */

struct orc_ras {
    int64_t n;
    int64_t nsub;
    int64_t *owner;       /* per cell: owning subdomain */
    int64_t *sub_ptr;     /* nsub+1 into sub_cells */
    int64_t *sub_cells;   /* cells of each Omega_s, ascending global index */
    orc_ilu **local;      /* ILU(0) of each local matrix */
};

void orc_ras_free(orc_ras *R)
{
    if (!R) return;
    if (R->local)
        for (int64_t s = 0; s < R->nsub; ++s) orc_ilu_free(R->local[s]);
    free(R->local);
    free(R->owner);
    free(R->sub_ptr);
    free(R->sub_cells);
    free(R);
}

int64_t orc_ras_nsub(const orc_ras *R) { return R->nsub; }
int64_t orc_ras_sub_size(const orc_ras *R, int64_t s) { return R->sub_ptr[s + 1] - R->sub_ptr[s]; }
void orc_ras_sub_cells(const orc_ras *R, int64_t s, int64_t *cells)
{
    memcpy(cells, R->sub_cells + R->sub_ptr[s], (size_t)orc_ras_sub_size(R, s) * sizeof(int64_t));
}
void orc_ras_owner(const orc_ras *R, int64_t *owner) { memcpy(owner, R->owner, (size_t)R->n * sizeof(int64_t)); }

/* Box index of coordinate v when [0, len) is split into p nearly equal parts,
 * the first (len % p) parts one longer. */
static int64_t split_index(int64_t v, int64_t len, int64_t p)
{
    int64_t base = len / p, rem = len % p;
    int64_t big = rem * (base + 1);
    if (v < big) return v / (base + 1);
    return rem + (v - big) / base;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

int orc_ras_setup(const orc_bcsr *A, int32_t nx, int32_t ny, int32_t nz,
                  int32_t px, int32_t py, int32_t pz, int32_t overlap,
                  orc_ras **out, int64_t *bad_cell)
{
    return orc_ras_setup_k(A, nx, ny, nz, px, py, pz, overlap, 0, out, bad_cell);
}

/* the local solver of RAS: ILU(level) (kind 0) or ILUT(p, tol) (kind 1) */
static int ras_setup(const orc_bcsr *A, int32_t nx, int32_t ny, int32_t nz, int32_t px, int32_t py, int32_t pz,
                     int32_t overlap, int kind, int32_t level, int32_t p, double tol, orc_ras **out,
                     int64_t *bad_cell);

int orc_ras_setup_k(const orc_bcsr *A, int32_t nx, int32_t ny, int32_t nz,
                    int32_t px, int32_t py, int32_t pz, int32_t overlap, int32_t level,
                    orc_ras **out, int64_t *bad_cell)
{
    return ras_setup(A, nx, ny, nz, px, py, pz, overlap, 0, level, 0, 0.0, out, bad_cell);
}

int orc_ras_setup_ilut(const orc_bcsr *A, int32_t nx, int32_t ny, int32_t nz,
                       int32_t px, int32_t py, int32_t pz, int32_t overlap, int32_t p, double tol,
                       orc_ras **out, int64_t *bad_cell)
{
    if (!(tol >= 0.0)) return ORC_ERR_ARG;
    return ras_setup(A, nx, ny, nz, px, py, pz, overlap, 1, 0, p, tol, out, bad_cell);
}

static int ras_setup(const orc_bcsr *A, int32_t nx, int32_t ny, int32_t nz, int32_t px, int32_t py, int32_t pz,
                     int32_t overlap, int kind, int32_t level, int32_t p, double tol, orc_ras **out,
                     int64_t *bad_cell)
{
    if (!A || !out || px < 1 || py < 1 || pz < 1 || overlap < 0 || level < 0) return ORC_ERR_ARG;
    if (px > nx || py > ny || pz > nz) return ORC_ERR_ARG;
    const int64_t n = A->n;
    if (n != (int64_t)nx * ny * nz) return ORC_ERR_ARG;
    if (bad_cell) *bad_cell = -1;
    orc_ras *R = (orc_ras *)calloc(1, sizeof(orc_ras));
    if (!R) return ORC_ERR_OOM;
    R->n = n;
    R->nsub = (int64_t)px * py * pz;
    R->owner = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    R->sub_ptr = (int64_t *)calloc((size_t)(R->nsub + 1), sizeof(int64_t));
    R->local = (orc_ilu **)calloc((size_t)R->nsub, sizeof(orc_ilu *));
    int64_t *dist = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *g2l = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!R->owner || !R->sub_ptr || !R->local || !dist || !queue || !g2l) {
        free(dist); free(queue); free(g2l);
        orc_ras_free(R);
        return ORC_ERR_OOM;
    }
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t sx = split_index(i, nx, px), sy = split_index(j, ny, py), sz = split_index(k, nz, pz);
                R->owner[k * nx * ny + j * nx + i] = (sz * py + sy) * px + sx;
            }
    /* Omega_s: cells within matrix-graph distance <= overlap of the owned set
     * (breadth-first search over the sparsity pattern of A). */
    int64_t total = 0;
    int64_t **cells_of = (int64_t **)calloc((size_t)R->nsub, sizeof(int64_t *));
    int64_t *count_of = (int64_t *)calloc((size_t)R->nsub, sizeof(int64_t));
    if (!cells_of || !count_of) {
        free(dist); free(queue); free(g2l); free(cells_of); free(count_of);
        orc_ras_free(R);
        return ORC_ERR_OOM;
    }
    for (int64_t i = 0; i < n; ++i) dist[i] = -1;
    int rc = ORC_OK;
    for (int64_t s = 0; s < R->nsub && rc == ORC_OK; ++s) {
        int64_t head = 0, tail = 0;
        for (int64_t c = 0; c < n; ++c)
            if (R->owner[c] == s) { dist[c] = 0; queue[tail++] = c; }
        while (head < tail) {
            int64_t c = queue[head++];
            if (dist[c] >= overlap) continue;
            for (int64_t p = A->rowptr[c]; p < A->rowptr[c + 1]; ++p) {
                int64_t nb = A->col[p];
                if (dist[nb] < 0) { dist[nb] = dist[c] + 1; queue[tail++] = nb; }
            }
        }
        cells_of[s] = (int64_t *)malloc((size_t)(tail > 0 ? tail : 1) * sizeof(int64_t));
        if (!cells_of[s]) { rc = ORC_ERR_OOM; break; }
        memcpy(cells_of[s], queue, (size_t)tail * sizeof(int64_t));
        qsort(cells_of[s], (size_t)tail, sizeof(int64_t), cmp_i64);
        count_of[s] = tail;
        total += tail;
        for (int64_t q = 0; q < tail; ++q) dist[queue[q]] = -1;
    }
    if (rc == ORC_OK) {
        R->sub_cells = (int64_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int64_t));
        if (!R->sub_cells) rc = ORC_ERR_OOM;
    }
    if (rc == ORC_OK) {
        int64_t off = 0;
        for (int64_t s = 0; s < R->nsub; ++s) {
            R->sub_ptr[s] = off;
            memcpy(R->sub_cells + off, cells_of[s], (size_t)count_of[s] * sizeof(int64_t));
            off += count_of[s];
        }
        R->sub_ptr[R->nsub] = off;
    }
    for (int64_t s = 0; s < R->nsub; ++s) free(cells_of[s]);
    free(cells_of);
    free(count_of);
    /* local matrices A_s = A restricted to Omega_s rows and columns, factored by ILU(0) */
    for (int64_t i = 0; i < n; ++i) g2l[i] = -1;
    for (int64_t s = 0; s < R->nsub && rc == ORC_OK; ++s) {
        const int64_t *cs = R->sub_cells + R->sub_ptr[s];
        const int64_t m = orc_ras_sub_size(R, s);
        for (int64_t q = 0; q < m; ++q) g2l[cs[q]] = q;
        int64_t nnzb = 0;
        for (int64_t q = 0; q < m; ++q)
            for (int64_t p = A->rowptr[cs[q]]; p < A->rowptr[cs[q] + 1]; ++p)
                if (g2l[A->col[p]] >= 0) ++nnzb;
        orc_bcsr *As = bcsr_alloc(m, nnzb);
        if (!As) { rc = ORC_ERR_OOM; break; }
        int64_t pos = 0;
        for (int64_t q = 0; q < m; ++q) {
            As->rowptr[q] = pos;
            for (int64_t p = A->rowptr[cs[q]]; p < A->rowptr[cs[q] + 1]; ++p) {
                int64_t lc = g2l[A->col[p]];
                if (lc < 0) continue;
                As->col[pos] = lc;   /* ascending, since g2l is monotone */
                memcpy(As->val + 9 * pos, A->val + 9 * p, 9 * sizeof(double));
                ++pos;
            }
        }
        As->rowptr[m] = pos;
        int64_t bad = -1;
        rc = (kind == 0) ? orc_iluk(As, level, &R->local[s], &bad) : orc_ilut(As, p, tol, &R->local[s], &bad);
        if (rc != ORC_OK && bad_cell) *bad_cell = (bad >= 0) ? cs[bad] : -1;
        orc_bcsr_free(As);
        for (int64_t q = 0; q < m; ++q) g2l[cs[q]] = -1;
    }
    free(dist);
    free(queue);
    free(g2l);
    if (rc != ORC_OK) {
        orc_ras_free(R);
        return rc;
    }
    *out = R;
    return ORC_OK;
}

/* z = sum_s Rtilde_s^T (L_s U_s)^{-1} R_s r: restrict r to Omega_s, apply the
 * local ILU(0), write back only the cells that s owns. */
int orc_ras_apply(void *ctx, const double *r, double *z)
{
    const orc_ras *R = (const orc_ras *)ctx;
    int64_t maxm = 0;
    for (int64_t s = 0; s < R->nsub; ++s)
        if (orc_ras_sub_size(R, s) > maxm) maxm = orc_ras_sub_size(R, s);
    double *rl = (double *)malloc((size_t)(maxm > 0 ? maxm : 1) * 3 * sizeof(double));
    double *zl = (double *)malloc((size_t)(maxm > 0 ? maxm : 1) * 3 * sizeof(double));
    if (!rl || !zl) { free(rl); free(zl); return ORC_ERR_OOM; }
    for (int64_t s = 0; s < R->nsub; ++s) {
        const int64_t *cs = R->sub_cells + R->sub_ptr[s];
        const int64_t m = orc_ras_sub_size(R, s);
        for (int64_t q = 0; q < m; ++q)
            for (int c = 0; c < 3; ++c) rl[3 * q + c] = r[3 * cs[q] + c];
        orc_ilu_apply(R->local[s], rl, zl);
        for (int64_t q = 0; q < m; ++q)
            if (R->owner[cs[q]] == s)
                for (int c = 0; c < 3; ++c) z[3 * cs[q] + c] = zl[3 * q + c];
    }
    free(rl);
    free(zl);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Krylov methods                                                       */
/* ------------------------------------------------------------------ */

static int has_nonfinite(int64_t n, const double *v)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 1;
    return 0;
}

static int apply_pc(orc_apply_fn pc, void *ctx, int64_t N, const double *in, double *out)
{
    if (!pc) {
        memcpy(out, in, (size_t)N * sizeof(double));
        return ORC_OK;
    }
    return pc(ctx, in, out);
}

/* The operator a Krylov method multiplies by: y = A x on vectors of length N
 * (the 3x3-block matrices here, the scalar matrices of scalar.c). */
typedef struct {
    int64_t N;
    orc_mv_fn mv;
    const void *ctx;
} orc_op;

static void bcsr_mv(const void *ctx, const double *x, double *y) { orc_spmv((const orc_bcsr *)ctx, x, y); }

/* r = b - A x; returns ||r|| */
static double true_residual(const orc_op *A, const double *b, const double *x, double *r, int64_t N)
{
    A->mv(A->ctx, x, r);
    for (int64_t i = 0; i < N; ++i) r[i] = b[i] - r[i];
    return orc_nrm2(N, r);
}

/* Classical Gram-Schmidt applied twice against V[0..j]; accumulates the
 * projection coefficients into h[0..j]. */
static void cgs2(int64_t N, double *const *V, int j, double *w, double *h)
{
    for (int i = 0; i <= j; ++i) h[i] = 0.0;
    double c[64];
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i <= j; ++i) c[i] = orc_dot(N, V[i], w);
        for (int i = 0; i <= j; ++i) {
            for (int64_t t = 0; t < N; ++t) w[t] -= c[i] * V[i][t];
            h[i] += c[i];
        }
    }
}

/* Apply previous rotations to column h[0..j+1], then form the rotation that
 * zeroes h[j+1]; updates g[j], g[j+1]. */
static void givens_step(int j, double *h, double *cs, double *sn, double *g)
{
    for (int i = 0; i < j; ++i) {
        double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
    }
    double a = h[j], b = h[j + 1];
    double rr = hypot(a, b);
    /* an all-zero column adds nothing to the Krylov space: rotate so that the
     * least-squares residual estimate stays |g_j| instead of dropping to 0 */
    double c = 0.0, s = 1.0;
    if (rr > 0.0) { c = a / rr; s = b / rr; }
    cs[j] = c;
    sn[j] = s;
    h[j] = rr;
    h[j + 1] = 0.0;
    g[j + 1] = -s * g[j];
    g[j] = c * g[j];
}

typedef struct {
    int flexible;          /* FGMRES: keep z_j in Z */
    orc_apply_fn fb;       /* fallback preconditioner (FGMRES) */
    void *fb_ctx;
    double theta;
} gm_opts;

static int gmres_core(const orc_op *A, orc_apply_fn pc, void *pc_ctx, const gm_opts *o,
                      const double *b, double *x, int32_t m, double tol, int64_t maxit,
                      orc_stats *st, double *hist)
{
    if (!A || !b || !x || m < 1 || m > 62 || maxit < 0) return ORC_ERR_ARG;
    const int64_t N = A->N;
    orc_stats dummy;
    if (!st) st = &dummy;
    st->its = 0; st->restarts = 0; st->fallbacks = 0; st->final_relres = 0.0; st->bad_cell = -1;
    if (has_nonfinite(N, b) || has_nonfinite(N, x)) return ORC_ERR_NAN;
    const double nb = orc_nrm2(N, b);
    if (nb == 0.0) {
        memset(x, 0, (size_t)N * sizeof(double));
        if (hist) hist[0] = 0.0;
        return ORC_OK;
    }
    double **V = (double **)calloc((size_t)(m + 1), sizeof(double *));
    double **Z = (double **)calloc((size_t)(m + 1), sizeof(double *));
    double *r = (double *)malloc((size_t)N * sizeof(double));
    double *w = (double *)malloc((size_t)N * sizeof(double));
    double *z = (double *)malloc((size_t)N * sizeof(double));
    double *u = (double *)malloc((size_t)N * sizeof(double));
    int rc = ORC_OK;
    if (!V || !Z || !r || !w || !z || !u) rc = ORC_ERR_OOM;
    for (int i = 0; i <= m && rc == ORC_OK; ++i) {
        V[i] = (double *)malloc((size_t)N * sizeof(double));
        if (!V[i]) rc = ORC_ERR_OOM;
        if (o->flexible) {
            Z[i] = (double *)malloc((size_t)N * sizeof(double));
            if (!Z[i]) rc = ORC_ERR_OOM;
        }
    }
    double H[64][64];   /* H[col][row] */
    double cs[64] = {0}, sn[64] = {0}, g[65] = {0}, y[64] = {0};
    int64_t its = 0;
    while (rc == ORC_OK) {
        double beta = true_residual(A, b, x, r, N);
        double relres = beta / nb;
        if (!isfinite(relres)) { rc = ORC_ERR_NAN; break; }
        if (its == 0 && hist) hist[0] = relres;
        st->final_relres = relres;
        if (relres <= tol) { rc = ORC_OK; break; }
        if (its >= maxit) { rc = ORC_NOT_CONVERGED; break; }
        for (int64_t t = 0; t < N; ++t) V[0][t] = r[t] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int jdone = 0;
        int consecutive_fb = 0, fb_rest = 0;
        for (int j = 0; j < m; ++j) {
            double hcol[65], cs_save[64], sn_save[64], g_save[65];
            int used_fb = 0, happy = 0;
            memcpy(cs_save, cs, sizeof(cs));
            memcpy(sn_save, sn, sizeof(sn));
            memcpy(g_save, g, sizeof(g));
            for (int attempt = 0; attempt < 2; ++attempt) {
                int want_fb = o->flexible && (fb_rest || attempt == 1);
                int prc;
                if (want_fb) {
                    prc = apply_pc(o->fb, o->fb_ctx, N, V[j], z);
                    used_fb = 1;
                } else {
                    prc = apply_pc(pc, pc_ctx, N, V[j], z);
                    if (o->flexible && (prc != ORC_OK || has_nonfinite(N, z))) {
                        continue;   /* discard, recompute with the fallback */
                    }
                }
                if (prc != ORC_OK) { rc = prc; break; }
                A->mv(A->ctx, z, w);
                double wnorm0 = orc_nrm2(N, w);
                cgs2(N, V, j, w, hcol);
                double hn = orc_nrm2(N, w);
                hcol[j + 1] = hn;
                memcpy(cs, cs_save, sizeof(cs));
                memcpy(sn, sn_save, sizeof(sn));
                memcpy(g, g_save, sizeof(g));
                givens_step(j, hcol, cs, sn, g);
                if (o->flexible && !want_fb && fabs(g[j + 1]) > o->theta * fabs(g_save[j])) {
                    continue;       /* failed to reduce the residual estimate */
                }
                for (int i = 0; i <= j + 1; ++i) H[j][i] = hcol[i];
                if (hn > 0.0)
                    for (int64_t t = 0; t < N; ++t) V[j + 1][t] = w[t] / hn;
                else
                    memset(V[j + 1], 0, (size_t)N * sizeof(double));
                if (o->flexible) memcpy(Z[j], z, (size_t)N * sizeof(double));
                happy = (hn <= 1e-14 * wnorm0);   /* happy breakdown */
                break;
            }
            if (rc != ORC_OK) break;
            if (o->flexible) {
                if (used_fb) { st->fallbacks++; consecutive_fb++; } else consecutive_fb = 0;
                if (consecutive_fb >= 3) fb_rest = 1;
            }
            ++its;
            jdone = j + 1;
            double est = fabs(g[j + 1]) / nb;
            if (hist) hist[its] = est;
            if (!isfinite(est)) { rc = ORC_ERR_NAN; break; }
            if (est <= tol || its >= maxit || happy) break;
        }
        if (rc != ORC_OK) break;
        /* y = H(0:jdone,0:jdone)^{-1} g, upper triangular back substitution */
        for (int i = jdone - 1; i >= 0; --i) {
            double s = g[i];
            for (int q = i + 1; q < jdone; ++q) s -= H[q][i] * y[q];
            y[i] = (H[i][i] != 0.0) ? s / H[i][i] : 0.0;
        }
        if (o->flexible) {
            for (int i = 0; i < jdone; ++i)
                for (int64_t t = 0; t < N; ++t) x[t] += y[i] * Z[i][t];
        } else {
            memset(u, 0, (size_t)N * sizeof(double));
            for (int i = 0; i < jdone; ++i)
                for (int64_t t = 0; t < N; ++t) u[t] += y[i] * V[i][t];
            int prc = apply_pc(pc, pc_ctx, N, u, z);
            if (prc != ORC_OK) { rc = prc; break; }
            for (int64_t t = 0; t < N; ++t) x[t] += z[t];
        }
        st->restarts++;
    }
    st->its = its;
    if (V) for (int i = 0; i <= m; ++i) free(V[i]);
    if (Z) for (int i = 0; i <= m; ++i) free(Z[i]);
    free(V); free(Z); free(r); free(w); free(z); free(u);
    return rc;
}

int orc_gmres(const orc_bcsr *A, orc_apply_fn pc, void *pc_ctx,
              const double *b, double *x, int32_t m, double tol, int64_t maxit,
              orc_stats *st, double *hist)
{
    if (!A) return ORC_ERR_ARG;
    gm_opts o = {0, NULL, NULL, 0.0};
    const orc_op op = {3 * A->n, bcsr_mv, A};
    return gmres_core(&op, pc, pc_ctx, &o, b, x, m, tol, maxit, st, hist);
}

int orc_gmres_op(int64_t N, orc_mv_fn mv, const void *mv_ctx, orc_apply_fn pc, void *pc_ctx,
                 const double *b, double *x, int32_t m, double tol, int64_t maxit, orc_stats *st, double *hist)
{
    if (N < 1 || !mv) return ORC_ERR_ARG;
    gm_opts o = {0, NULL, NULL, 0.0};
    const orc_op op = {N, mv, mv_ctx};
    return gmres_core(&op, pc, pc_ctx, &o, b, x, m, tol, maxit, st, hist);
}

int orc_fgmres(const orc_bcsr *A, orc_apply_fn pc, void *pc_ctx,
               orc_apply_fn fb, void *fb_ctx, double theta,
               const double *b, double *x, int32_t m, double tol, int64_t maxit,
               orc_stats *st, double *hist)
{
    gm_opts o = {1, fb, fb_ctx, theta};
    if (!fb || !A) return ORC_ERR_ARG;
    const orc_op op = {3 * A->n, bcsr_mv, A};
    return gmres_core(&op, pc, pc_ctx, &o, b, x, m, tol, maxit, st, hist);
}

static int bicgstab_core(const orc_op *A, orc_apply_fn pc, void *pc_ctx,
                         const double *b, double *x, double tol, int64_t maxit,
                         orc_stats *st, double *hist)
{
    if (!A || !b || !x || maxit < 0) return ORC_ERR_ARG;
    const int64_t N = A->N;
    orc_stats dummy;
    if (!st) st = &dummy;
    st->its = 0; st->restarts = 0; st->fallbacks = 0; st->final_relres = 0.0; st->bad_cell = -1;
    if (has_nonfinite(N, b) || has_nonfinite(N, x)) return ORC_ERR_NAN;
    const double nb = orc_nrm2(N, b);
    if (nb == 0.0) {
        memset(x, 0, (size_t)N * sizeof(double));
        if (hist) hist[0] = 0.0;
        return ORC_OK;
    }
    double *r = (double *)malloc((size_t)N * sizeof(double));
    double *rh = (double *)malloc((size_t)N * sizeof(double));
    double *p = (double *)calloc((size_t)N, sizeof(double));
    double *v = (double *)calloc((size_t)N, sizeof(double));
    double *ph = (double *)malloc((size_t)N * sizeof(double));
    double *s = (double *)malloc((size_t)N * sizeof(double));
    double *sh = (double *)malloc((size_t)N * sizeof(double));
    double *t = (double *)malloc((size_t)N * sizeof(double));
    int rc = ORC_OK;
    if (!r || !rh || !p || !v || !ph || !s || !sh || !t) rc = ORC_ERR_OOM;
    int64_t its = 0;
    int done = 0;
    if (rc == ORC_OK) {
        double rn = true_residual(A, b, x, r, N);
        st->final_relres = rn / nb;
        if (hist) hist[0] = rn / nb;
        if (!isfinite(rn)) rc = ORC_ERR_NAN;
        else if (rn / nb <= tol) done = 1;
    }
    if (rc == ORC_OK && !done) {
        memcpy(rh, r, (size_t)N * sizeof(double));
        double rho = 1.0, alpha = 1.0, omega = 1.0;
        const double nrh = orc_nrm2(N, rh);
        for (;;) {
            if (its >= maxit) { rc = ORC_NOT_CONVERGED; break; }
            double rho_new = orc_dot(N, rh, r);
            if (!(fabs(rho_new) >= 1e-300 * nrh * orc_nrm2(N, r))) { rc = ORC_BREAKDOWN; break; }
            double beta = (rho_new / rho) * (alpha / omega);
            for (int64_t q = 0; q < N; ++q) p[q] = r[q] + beta * (p[q] - omega * v[q]);
            rc = apply_pc(pc, pc_ctx, N, p, ph);
            if (rc != ORC_OK) break;
            A->mv(A->ctx, ph, v);
            double rv = orc_dot(N, rh, v);
            if (rv == 0.0 || !isfinite(rv)) { rc = isfinite(rv) ? ORC_BREAKDOWN : ORC_ERR_NAN; break; }
            alpha = rho_new / rv;
            for (int64_t q = 0; q < N; ++q) s[q] = r[q] - alpha * v[q];
            double sn = orc_nrm2(N, s);
            if (sn / nb <= tol) {
                for (int64_t q = 0; q < N; ++q) x[q] += alpha * ph[q];
                ++its;
                double rn = true_residual(A, b, x, r, N);
                if (hist) hist[its] = rn / nb;
                st->final_relres = rn / nb;
                if (rn / nb <= tol) { rc = ORC_OK; break; }
                rho = rho_new;
                continue;   /* r now holds the recomputed residual */
            }
            rc = apply_pc(pc, pc_ctx, N, s, sh);
            if (rc != ORC_OK) break;
            A->mv(A->ctx, sh, t);
            double tt = orc_dot(N, t, t);
            double ts = orc_dot(N, t, s);
            omega = (tt > 0.0) ? ts / tt : 0.0;
            for (int64_t q = 0; q < N; ++q) x[q] += alpha * ph[q] + omega * sh[q];
            for (int64_t q = 0; q < N; ++q) r[q] = s[q] - omega * t[q];
            rho = rho_new;
            ++its;
            double rn = orc_nrm2(N, r);
            if (hist) hist[its] = rn / nb;
            if (!isfinite(rn)) { rc = ORC_ERR_NAN; break; }
            if (rn / nb <= tol) {
                double tr = true_residual(A, b, x, r, N);
                st->final_relres = tr / nb;
                if (tr / nb <= tol) { rc = ORC_OK; break; }
            }
            if (omega == 0.0) { rc = ORC_BREAKDOWN; break; }
        }
    }
    st->its = its;
    if (rc != ORC_ERR_OOM) {
        double tr = true_residual(A, b, x, r, N);
        st->final_relres = tr / nb;
    }
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t);
    return rc;
}

int orc_bicgstab(const orc_bcsr *A, orc_apply_fn pc, void *pc_ctx,
                 const double *b, double *x, double tol, int64_t maxit,
                 orc_stats *st, double *hist)
{
    if (!A) return ORC_ERR_ARG;
    const orc_op op = {3 * A->n, bcsr_mv, A};
    return bicgstab_core(&op, pc, pc_ctx, b, x, tol, maxit, st, hist);
}

int orc_bicgstab_op(int64_t N, orc_mv_fn mv, const void *mv_ctx, orc_apply_fn pc, void *pc_ctx,
                    const double *b, double *x, double tol, int64_t maxit, orc_stats *st, double *hist)
{
    if (N < 1 || !mv) return ORC_ERR_ARG;
    const orc_op op = {N, mv, mv_ctx};
    return bicgstab_core(&op, pc, pc_ctx, b, x, tol, maxit, st, hist);
}
