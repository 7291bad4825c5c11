/*
 * CPU ORACLE -- test infrastructure only.
 *
 * A plain, serial, FP64 implementation of what the GPU solver computes, used
 * to check it.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg may load it; the product path never does.  It shares no code
 * with the GPU library: its own storage (block CSR), its own generic IKJ
 * ILU(0), its own Krylov drivers.
 *
 * What each routine follows:
 *  - operations y = A x, <x,y>, ||x||: the paper's "Algebraic Operations"
 *    subsection (distributed matrices and vectors);
 *  - ILU: "LU x = b <=> L y = b, U x = y" solved row by row (Preconditioners,
 *    Restricted Additive Schwarz subsection), with ILU(0) as the default local
 *    solver (RAS default-parameter figure); the factorisation is the textbook
 *    IKJ ILU(0) (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
 *    sec. 10.3) with 3x3 blocks, divides replaced by right-multiplication by
 *    the pivot block's inverse;
 *  - RAS: restricted additive Schwarz of Cai & Sarkis (1999), the paper's
 *    [DDM] citation, overlap 1 by default;
 *  - GMRES(m): Saad & Schultz (1986), right preconditioned, classical
 *    Gram-Schmidt applied twice, Givens rotations;
 *  - BiCGSTAB: van der Vorst (1992), right preconditioned;
 *  - FGMRES: Saad (1993), with a fallback preconditioner.
 * Parity status of each routine is recorded in the tests that pin it.
 */
#ifndef RSV_ORACLE_H
#define RSV_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_OK = 0,
    ORC_NOT_CONVERGED = 1,
    ORC_BREAKDOWN = 2,
    ORC_ERR_ARG = -1,
    ORC_ERR_OOM = -2,
    ORC_ERR_ZERO_PIVOT = -4,
    ORC_ERR_NAN = -5,
    ORC_ERR_PATTERN = -6,
};

/* Block CSR, 3x3 blocks stored row-major, columns ascending in each row. */
typedef struct orc_bcsr {
    int64_t n;        /* block rows */
    int64_t nnzb;
    int64_t *rowptr;  /* n+1 */
    int64_t *col;     /* nnzb */
    double  *val;     /* 9*nnzb */
} orc_bcsr;

typedef int (*orc_apply_fn)(void *ctx, const double *in, double *out);
typedef void (*orc_mv_fn)(const void *ctx, const double *x, double *y);   /* y = A x */

typedef struct orc_stats {
    int64_t its;         /* Arnoldi steps (GMRES/FGMRES) or iterations (BiCGSTAB) */
    int64_t restarts;    /* completed GMRES cycles */
    int64_t fallbacks;   /* FGMRES columns recomputed with the fallback */
    double  final_relres;/* recomputed ||b - A x|| / ||b|| */
    int64_t bad_cell;    /* block row of a zero pivot, else -1 */
} orc_stats;

/* ---- storage ---- */
int  orc_bcsr_from_stencil(int32_t nx, int32_t ny, int32_t nz, const double *blocks, orc_bcsr **out);
int  orc_bcsr_from_dense_pattern(int64_t n, const int64_t *rowptr, const int64_t *col, const double *val, orc_bcsr **out);
void orc_bcsr_free(orc_bcsr *A);
int64_t orc_bcsr_nnzb(const orc_bcsr *A);
/* copy out rowptr/col/val (sizes n+1, nnzb, 9*nnzb) */
void orc_bcsr_export(const orc_bcsr *A, int64_t *rowptr, int64_t *col, double *val);

/* ---- algebraic operations ---- */
void   orc_spmv(const orc_bcsr *A, const double *x, double *y);            /* y = A x */
double orc_dot(int64_t n, const double *x, const double *y);
double orc_nrm2(int64_t n, const double *x);

/* ---- ILU(0) ---- */
typedef struct orc_ilu orc_ilu;
int  orc_ilu0(const orc_bcsr *A, orc_ilu **out, int64_t *bad_cell);
void orc_ilu_free(orc_ilu *F);
const orc_bcsr *orc_ilu_factors(const orc_ilu *F);   /* strict lower = L, upper incl. diagonal = U */
int  orc_ilu_apply(void *F, const double *r, double *z);    /* z = (LU)^{-1} r */
/* ILU(k): the IKJ factorisation on the level-k fill pattern (k = 0: ILU(0)) */
int  orc_iluk(const orc_bcsr *A, int32_t k, orc_ilu **out, int64_t *bad_cell);
/* the level-k pattern (rowptr n+1, col and level nnzb entries when nnzb <= cap); returns nnzb */
int  orc_iluk_pattern(const orc_bcsr *A, int32_t k, int64_t *rowptr, int64_t *col, int64_t *level, int64_t cap);
int  orc_ilu_apply_f32(void *F, const double *r, double *z);/* FP32 factors + FP32 sweeps */
/* ILUT(p, tol) with 3x3 blocks (ilut.c); p < 0: per row, as many blocks in
 * each triangle as that triangle of A's row holds */
int  orc_ilut(const orc_bcsr *A, int32_t p, double tol, orc_ilu **out, int64_t *bad_cell);
/* wrap finished factors (takes LU over), and a zeroed block CSR */
int  orc_ilu_wrap(orc_bcsr *LU, orc_ilu **out, int64_t *bad_cell);
orc_bcsr *orc_bcsr_new(int64_t n, int64_t nnzb);

/* ---- RAS ---- */
typedef struct orc_ras orc_ras;
int  orc_ras_setup(const orc_bcsr *A, int32_t nx, int32_t ny, int32_t nz,
                   int32_t px, int32_t py, int32_t pz, int32_t overlap,
                   orc_ras **out, int64_t *bad_cell);
/* the same with ILU(level) local solvers */
int  orc_ras_setup_k(const orc_bcsr *A, int32_t nx, int32_t ny, int32_t nz,
                     int32_t px, int32_t py, int32_t pz, int32_t overlap, int32_t level,
                     orc_ras **out, int64_t *bad_cell);
/* the same with ILUT(p, tol) local solvers */
int  orc_ras_setup_ilut(const orc_bcsr *A, int32_t nx, int32_t ny, int32_t nz,
                        int32_t px, int32_t py, int32_t pz, int32_t overlap, int32_t p, double tol,
                        orc_ras **out, int64_t *bad_cell);
void orc_ras_free(orc_ras *R);
int  orc_ras_apply(void *R, const double *r, double *z);
int64_t orc_ras_nsub(const orc_ras *R);
int64_t orc_ras_sub_size(const orc_ras *R, int64_t s);           /* |Omega_s| */
void orc_ras_sub_cells(const orc_ras *R, int64_t s, int64_t *cells); /* ascending */
void orc_ras_owner(const orc_ras *R, int64_t *owner);            /* per cell */

/* ---- Krylov ---- */
int orc_gmres(const orc_bcsr *A, orc_apply_fn pc, void *pc_ctx,
              const double *b, double *x, int32_t m, double tol, int64_t maxit,
              orc_stats *st, double *hist /* nullable, length maxit+1 */);
int orc_bicgstab(const orc_bcsr *A, orc_apply_fn pc, void *pc_ctx,
                 const double *b, double *x, double tol, int64_t maxit,
                 orc_stats *st, double *hist);
int orc_fgmres(const orc_bcsr *A, orc_apply_fn pc, void *pc_ctx,
               orc_apply_fn fb, void *fb_ctx, double theta,
               const double *b, double *x, int32_t m, double tol, int64_t maxit,
               orc_stats *st, double *hist);

/* the same Krylov methods for any operator y = A x on vectors of length N */
int orc_gmres_op(int64_t N, orc_mv_fn mv, const void *mv_ctx, orc_apply_fn pc, void *pc_ctx,
                 const double *b, double *x, int32_t m, double tol, int64_t maxit, orc_stats *st, double *hist);
int orc_bicgstab_op(int64_t N, orc_mv_fn mv, const void *mv_ctx, orc_apply_fn pc, void *pc_ctx,
                    const double *b, double *x, double tol, int64_t maxit, orc_stats *st, double *hist);

/* ---- scalar (one unknown per cell) systems, scalar.c ---- */
typedef struct orc_csr orc_csr;
typedef struct orc_silu orc_silu;
typedef struct orc_sras orc_sras;
int  orc_csr_from_stencil(int32_t nx, int32_t ny, int32_t nz, const double *coef /* [n][7] */, orc_csr **out);
void orc_csr_free(orc_csr *A);
int64_t orc_csr_nnz(const orc_csr *A);
void orc_csr_export(const orc_csr *A, int64_t *rowptr, int64_t *col, double *val);
void orc_csr_spmv(const orc_csr *A, const double *x, double *y);
/* a copy of rowptr (n+1) / col / val; columns strictly ascending in each row */
int  orc_csr_from_arrays(int64_t n, const int64_t *rowptr, const int64_t *col, const double *val, orc_csr **out);
/* read-only views of the arrays (owned by A) */
void orc_csr_view(const orc_csr *A, int64_t *n, const int64_t **rowptr, const int64_t **col, const double **val);
int  orc_csr_ilu0(const orc_csr *A, orc_silu **out, int64_t *bad_row);
void orc_silu_free(orc_silu *F);
const orc_csr *orc_silu_factors(const orc_silu *F);
int  orc_silu_apply(void *F, const double *r, double *z);
int  orc_sras_setup(const orc_csr *A, int32_t nx, int32_t ny, int32_t nz, int32_t px, int32_t py, int32_t pz,
                    int32_t overlap, orc_sras **out, int64_t *bad_row);
void orc_sras_free(orc_sras *R);
int64_t orc_sras_nsub(const orc_sras *R);
int64_t orc_sras_sub_size(const orc_sras *R, int64_t s);
void orc_sras_sub_cells(const orc_sras *R, int64_t s, int64_t *cells);
int  orc_sras_apply(void *R, const double *r, double *z);
int  orc_csr_gmres(const orc_csr *A, orc_apply_fn pc, void *pc_ctx, const double *b, double *x, int32_t m,
                   double tol, int64_t maxit, orc_stats *st, double *hist);
int  orc_csr_bicgstab(const orc_csr *A, orc_apply_fn pc, void *pc_ctx, const double *b, double *x, double tol,
                      int64_t maxit, orc_stats *st, double *hist);

/* ---- aggregation multigrid V-cycle for 7-point scalar systems (mg.c) ---- */
typedef struct orc_mg orc_mg;
int  orc_mg_setup(const orc_csr *A /* not copied; must outlive */, int32_t nx, int32_t ny, int32_t nz,
                  int32_t coarse_max, int32_t pre, int32_t post, orc_mg **out);
void orc_mg_free(orc_mg *M);
int  orc_mg_apply(void *M, const double *b, double *x);       /* x = one V-cycle from 0 */
int32_t orc_mg_levels(const orc_mg *M);
void orc_mg_level_dims(const orc_mg *M, int32_t l, int32_t *dims);
const orc_csr *orc_mg_level_matrix(const orc_mg *M, int32_t l);
int  orc_mg_gs_sweep(const orc_mg *M, const double *b, double *x, int32_t colour);   /* level 0 */

/* ---- CPR-type two-stage preconditioners (cpr.c) ---- */
enum { ORC_CPR_FP = 0, ORC_CPR_PF = 1, ORC_CPR_FPF = 2, ORC_CPR_FFPF = 3 };
enum { ORC_DECOUPLE_NONE = 0, ORC_DECOUPLE_QUASI_IMPES = 1, ORC_DECOUPLE_ABF = 2 };
typedef struct orc_cpr orc_cpr;
int  orc_cpr_setup(const orc_bcsr *A /* not copied */, int32_t nx, int32_t ny, int32_t nz, int32_t variant,
                   int32_t decouple, orc_apply_fn R, void *R_ctx, int32_t coarse_max, int32_t pre, int32_t post,
                   orc_cpr **out, int64_t *bad_cell);
void orc_cpr_free(orc_cpr *P);
int  orc_cpr_apply(void *P, const double *f, double *x);
void orc_cpr_weights(const orc_cpr *P, double *w);                /* [n][3] */
const orc_csr *orc_cpr_pressure_matrix(const orc_cpr *P);
const orc_mg *orc_cpr_mg(const orc_cpr *P);

/* ---- learned preconditioner network (unet.c) ---- */
double  orc_bf16(double x);      /* round to the nearest BF16 value (ties to even) */
void    orc_conv3d_fwd(int nx, int ny, int nz, int cin, int cout, const double *x, const double *w,
                       const double *b, double *y);
void    orc_conv3d_bwd(int nx, int ny, int nz, int cin, int cout, const double *x, const double *w,
                       const double *dy, double *dx, double *dw, double *db);
int64_t orc_unet_nparams(int c0, int c1, int c2);
int     orc_unet_forward(int c0, int c1, int c2, int nx, int ny, int nz, const double *params,
                         const double *x0, double *y, int emulate_bf16);
int     orc_unet_loss_grad(int c0, int c1, int c2, int nx, int ny, int nz, const double *params,
                           const double *x0, const double *target, double *grad, double *loss, int emulate_bf16);
double  orc_unet_prepare(int nx, int ny, int nz, const double *r, const double *lnk, double *x0);
void    orc_adam(int64_t n, double *p, const double *g, double *m, double *v, int64_t t, double lr);

/* ---- Hilbert space-filling-curve partition (hsfc.c) ---- */
int orc_hsfc_key3(const double *c, int32_t levels, uint64_t *key);        /* c in [0,1]^3, levels 1..21 */
int orc_hsfc_grid_keys(int32_t nx, int32_t ny, int32_t nz, int32_t levels, uint64_t *keys);
int orc_hsfc_partition(int64_t n, const uint64_t *keys, int32_t nparts, int32_t *part);
int orc_partition_quality(int32_t nx, int32_t ny, int32_t nz, const int32_t *part, int32_t nparts, double *q,
                          int64_t *per_part);

/* plain dense 3x3 helpers exposed for the pins */
int orc_inv3(const double *a, double *ainv);  /* LU with partial pivoting; 0 ok, -4 singular */

#ifdef __cplusplus
}
#endif
#endif
