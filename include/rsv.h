/*
 * rsv -- preconditioned Krylov solver for 3x3-block, 7-point-stencil
 * reservoir Jacobians on one MI355X (gfx950).  C ABI.
 *
 * The calls follow the paper's problem statement (arxiv 1602.05901):
 * a structured grid nx*ny*nz (Grid section), a cell -> row map (MAP section),
 * an assembled block matrix (Distributed Matrices and Vectors section), a
 * preconditioner with setup / apply / destroy hooks (Preconditioners section,
 * SOLVER_PC and PC_TYPE figures) and a solver with rtol / maxit / restart
 * (Solvers section, SOLVER figure).
 *
 * Conventions (every call):
 *  - Every call returns an rsv_status.  RSV_OK = 0; positive values are
 *    warnings whose outputs are still filled; negative values are errors.
 *    No C++ exception crosses this boundary.
 *  - The caller owns every buffer it passes.  Handles own their device
 *    memory until the matching *_destroy.  Destroy in the order
 *    precond -> matrix -> grid -> net -> ctx.
 *  - Vectors are FP64, contiguous, length 3*ncell, in block-row order with
 *    the three unknowns of a cell interleaved (row = 3*block_row + comp).
 *    Vector pointers are DEVICE pointers unless a call says otherwise.
 *  - All device work is enqueued on the context's stream (rsv_set_stream);
 *    calls that return scalars synchronise that stream before returning.
 *  - A context is used by one host thread at a time.
 */
#ifndef RSV_H
#define RSV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rsv_status;
enum {
    RSV_OK = 0,
    RSV_NOT_CONVERGED = 1,   /* maxit reached: x holds the last iterate, stats filled */
    RSV_BREAKDOWN = 2,       /* BiCGSTAB rho = 0 or omega = 0: x holds the current iterate */
    RSV_ERR_ARG = -1,        /* invalid argument (null handle, bad size, bad enum) */
    RSV_ERR_OOM = -2,        /* device or host allocation failed */
    RSV_ERR_HIP = -3,        /* a HIP runtime call failed (rsv_last_error has the text) */
    RSV_ERR_ZERO_PIVOT = -4, /* singular or near-singular 3x3 pivot; stats.bad_cell names it */
    RSV_ERR_NAN = -5,        /* NaN/Inf in the right-hand side, x0 or a recurrence */
    RSV_ERR_PATTERN = -6,    /* nonzero block in a stencil slot whose neighbour is outside the grid */
    RSV_ERR_TIMEOUT = -7     /* a wavefront kernel's bounded wait expired (should not happen) */
};

typedef enum {
    RSV_BOTTOM_UP = 0,   /* block_row = nx*ny*k + nx*j + i (Grid section, default numbering) */
    RSV_TOP_DOWN = 1     /* block_row = nx*ny*(nz-1-k) + nx*j + i (the top-to-bottom numbering,
                            read with nz-1-k so that rows stay in [0, ncell)) */
} rsv_ordering;

typedef enum { RSV_MEM_HOST = 0, RSV_MEM_DEVICE = 1 } rsv_mem;

/* Preconditioner kinds; mirrors the paper's PC_TYPE (RAS, ..., USER, NON). */
typedef enum {
    RSV_PC_NONE = 0,
    RSV_PC_BILU0 = 1,    /* global block ILU(0) in natural (bottom-up) order */
    RSV_PC_RAS = 2,      /* restricted additive Schwarz, local block ILU(0) */
    RSV_PC_LEARNED = 3,  /* user-type preconditioner: the U-Net, BILU0 fallback (FGMRES only) */
    RSV_PC_CPR = 4       /* CPR-type two-stage preconditioner (the paper's CPR_FP .. CPR_FFPF) */
} rsv_pc_type;

/* The four CPR-type algorithms of the CPR-like Preconditioners subsection.
 * R = the whole-system stage (RAS or BILU0), P = the pressure stage
 * x += Pi_p M_g(A_pp)^-1 Pi_r W r, each stage applied to the current residual
 * r = f - A x:
 *   RSV_CPR_FP    x = R f, then P;
 *   RSV_CPR_PF    x = Pi_p M_g^-1 Pi_r W f, then R (the printed steps
 *                 overwrite the first x and apply R to f again; read as the
 *                 two-stage form);
 *   RSV_CPR_FPF   x = R f, then P, then R (the simulator runs' choice);
 *   RSV_CPR_FFPF  x = R f, then R, then P, then R. */
typedef enum { RSV_CPR_FP = 0, RSV_CPR_PF = 1, RSV_CPR_FPF = 2, RSV_CPR_FFPF = 3 } rsv_cpr_variant;

/* Decoupling of the pressure equation (the simulator runs name a decoupling
 * without defining it).  The pressure equation of cell c is w_c^T times block
 * row c, A_pp(c, n) = w_c^T A_cn e_0, and the restricted residual is
 * w_c^T r_c; the pressure is unknown 0 of each cell.
 *   RSV_DECOUPLE_NONE         w_c = e_0: A_pp is the pressure-pressure submatrix;
 *   RSV_DECOUPLE_QUASI_IMPES  w_c = (1, w1, w2) with w_c^T A_cc zero in columns
 *                             1 and 2 (Scheichl, Masson & Wendebourg 2003);
 *   RSV_DECOUPLE_ABF          w_c^T = e_0^T A_cc^-1 (alternate block
 *                             factorisation, Bank, Chan, Coughran & Smith 1989). */
typedef enum { RSV_DECOUPLE_NONE = 0, RSV_DECOUPLE_QUASI_IMPES = 1, RSV_DECOUPLE_ABF = 2 } rsv_decouple;

typedef enum { RSV_FP64 = 0, RSV_FP32 = 1 } rsv_precision;

/* Local ILU of BILU0 and RAS (the RAS parameters' solver: ILUK or ILUT). */
typedef enum { RSV_LOCAL_ILUK = 0, RSV_LOCAL_ILUT = 1 } rsv_local_solver;

typedef enum { RSV_GMRES = 0, RSV_BICGSTAB = 1, RSV_FGMRES = 2 } rsv_method;

/* Orthogonalisation of the GMRES Arnoldi vectors.  RSV_CGS2: classical
 * Gram-Schmidt applied twice at every step (three passes over the basis).
 * RSV_DCGS2: the same two classical passes with the second one delayed by a
 * step (Bielich, Langou, Thomas, Swirydowicz, Yamazaki, Boman, Parallel
 * Computing 2022): one pass computes V^T [v_j, w], the next corrects v_j and
 * projects w (two passes over the basis, one reduction per step); the
 * Hessenberg column of the previous step is corrected on the host.  Both give
 * the GMRES iterates of the Linear System / Solvers section up to rounding.
 * FGMRES always uses RSV_CGS2. */
typedef enum { RSV_CGS2 = 0, RSV_DCGS2 = 1 } rsv_ortho;

typedef struct rsv_ctx rsv_ctx;
typedef struct rsv_grid rsv_grid;
typedef struct rsv_matrix rsv_matrix;
typedef struct rsv_precond rsv_precond;
typedef struct rsv_net rsv_net;

/* Preconditioner parameters.  Defaults (rsv_pc_params_default) follow the
 * paper's RAS default-parameter figure: overlap 1, ILU level 0. */
typedef struct rsv_pc_params {
    int32_t type;        /* rsv_pc_type */
    int32_t precision;   /* rsv_precision of the stored factors and triangular sweeps */
    int32_t ras_px, ras_py, ras_pz;  /* RAS: subdomain boxes per axis (default 4,4,4) */
    int32_t ras_overlap; /* RAS: matrix-graph overlap distance (default 1) */
    int32_t iluk_level;  /* level of fill k of the local ILU(k) (the RAS parameters' iluk_level, default 0):
                          * 0 = ILU(0) on the fast paths; 1..8 (3x3-block matrices, FP64) = ILU(k) by
                          * levels of fill, rows scheduled by dependency level, one workgroup per
                          * subdomain (type RAS: the local solver; type BILU0: the whole grid) */
    int32_t pipelined;   /* 1 (default): sync-free tiled wavefront sweeps (RAS: every subdomain's local
                          * system in one auxiliary grid of boxes, swept together); 0: BILU0 one launch
                          * per hyperplane, RAS one workgroup per subdomain (reference mappings) */
    rsv_net *net;        /* LEARNED: trained network (not owned) */
    const float *lnk;    /* LEARNED: DEVICE pointer, ln k per cell in block-row order (not copied; must outlive the precond) */
    double theta;        /* LEARNED: fallback when a step's residual estimate exceeds theta * previous (default 0.9, the
                            best of 0.99 / 0.9 / 0.8 / 0.5 on 64 held-out 64x64x32 systems at which the
                            network is still accepted on some columns) */
    int32_t learned_mode;/* LEARNED: 0 (default) z = s N(r/s); 1 z = t + s N(r1/s) with t = BILU0^-1 r,
                          * r1 = r - A t, s = rms(r1): the network corrects what one BILU0 step leaves */
    int32_t ras_stack;   /* RAS, pipelined: subdomain boxes stacked per tile column of the auxiliary
                          * grid (0, default: as many as keep four tiles per compute unit) */
    int32_t ras_group;   /* RAS, pipelined: boxes placed side by side in groups of ras_group x ras_group,
                          * each group padded to whole 8 x 8 tiles (0, default: 1, each box padded alone;
                          * at most 16; made smaller when the boxes of a layer do not fill a group) */
    /* CPR (3x3-block matrices).  The stage R is built from the fields above
     * with type cpr_stage (precision, RAS boxes and overlap, iluk_level,
     * pipelined apply to it).  M_g is one V-cycle of an aggregation multigrid
     * on the grid: 2x2x2 aggregates (an axis of one cell is kept), Galerkin
     * coarse operators (which stay 7-point), red-black Gauss-Seidel smoothing
     * (mg_pre sweeps red then black, mg_post sweeps black then red), and an
     * exact solve on the first level with at most mg_coarse cells.  With
     * precision RSV_FP32 the stage R sweeps in FP32 and the CPR's own
     * residual products and multigrid read FP32 copies of A and of the level
     * operators (arithmetic and vectors stay FP64). */
    int32_t cpr_variant; /* rsv_cpr_variant (default RSV_CPR_FPF) */
    int32_t cpr_stage;   /* RSV_PC_RAS (default) or RSV_PC_BILU0 */
    int32_t cpr_decouple;/* rsv_decouple (default RSV_DECOUPLE_NONE) */
    int32_t mg_pre;      /* pre-smoothing sweeps, 1..8 (default 1) */
    int32_t mg_post;     /* post-smoothing sweeps, 1..8 (default 1) */
    int32_t mg_coarse;   /* largest coarsest level, 1..1024 cells (default 128) */
    /* Local solver of BILU0 / RAS on 3x3-block matrices (the RAS parameters'
     * solver field): RSV_LOCAL_ILUK (default; ILU(iluk_level)) or
     * RSV_LOCAL_ILUT, threshold ILU with 3x3 blocks: row by row, the blocks
     * left of the diagonal are eliminated in ascending order and a block B of
     * the work row is dropped when |B|_F^2 < ilut_tol^2 x (sum of |A_ij|_F^2
     * over A's row); of the rest, the ilut_p largest on each side are kept
     * (ilut_p = -1: as many as A's row holds on that side; at most 32).
     * FP64 factors; one wavefront per subdomain factors on the device with
     * the work row in LDS (a subdomain's band, nx_s*ny_s cells, must fit:
     * else RSV_ERR_ARG), then the ILU(k) apply runs on the resulting
     * pattern.  A row whose work list outgrows 512 blocks gives RSV_ERR_ARG. */
    int32_t local_solver;/* rsv_local_solver */
    int32_t ilut_p;      /* default -1 */
    double ilut_tol;     /* default 1e-3 */
    int32_t reserved[4];
} rsv_pc_params;

/* Solver parameters; mirrors SOLVER (rtol, atol, maxit, restart). */
typedef struct rsv_solver_params {
    int32_t method;      /* rsv_method */
    int32_t restart;     /* GMRES/FGMRES cycle length m (default 30, max 60) */
    double tol;          /* stop when the recomputed ||b - A x||_2 / ||b||_2 <= tol (default 1e-8) */
    int64_t maxit;       /* Arnoldi steps (GMRES/FGMRES) or iterations (BiCGSTAB); default 10000 */
    double rtol;         /* optional, 0 = off: stop when ||r|| <= rtol * ||r0|| */
    double atol;         /* optional, 0 = off: stop when ||r|| <= atol */
    int32_t record_history;  /* 1: keep per-step residual estimates (rsv_solve_history) */
    int32_t ortho;       /* GMRES: rsv_ortho (default RSV_CGS2) */
    int32_t reserved[6];
} rsv_solver_params;

typedef struct rsv_stats {
    int64_t its;          /* Arnoldi steps or BiCGSTAB iterations performed */
    int64_t restarts;     /* completed GMRES cycles */
    int64_t fallbacks;    /* FGMRES columns computed with the fallback preconditioner */
    double final_relres;  /* recomputed ||b - A x|| / ||b|| at exit */
    double solve_ms;      /* wall time of the call (host clock, after the final sync) */
    int64_t bad_cell;     /* block row of a zero pivot, else -1 */
    int32_t status;       /* same as the return value */
    int32_t reserved;
} rsv_stats;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device_ordinal`; work goes to the null
 * stream until rsv_set_stream.  Errors: RSV_ERR_ARG (bad ordinal), RSV_ERR_HIP. */
rsv_status rsv_create(int32_t device_ordinal, rsv_ctx **out);
/* Enqueue all later work on `hip_stream` (a hipStream_t, e.g. torch's
 * current_stream().cuda_stream); NULL selects the null stream. */
rsv_status rsv_set_stream(rsv_ctx *ctx, void *hip_stream);
void rsv_destroy(rsv_ctx *ctx);
const char *rsv_status_str(rsv_status s);
/* Text of the last error recorded on ctx (empty string if none; ctx may be NULL). */
const char *rsv_last_error(const rsv_ctx *ctx);
/* ABI version: major*10000 + minor*100 + patch. */
int32_t rsv_version(void);
/* Device facts the solver sizes itself by, written to the HOST array info:
 * [0] compute units, [1] LDS bytes a workgroup may use, [2] LDS bytes per CU,
 * [3] ring depth of the forward FP64 sweep, [4] of the backward FP64 sweep.
 * Writes min(n, 5) entries.  Errors: RSV_ERR_ARG. */
rsv_status rsv_device_info(const rsv_ctx *ctx, int64_t *info, int32_t n);
/* Bound, in seconds, on every wait of the pipelined wavefront kernels (a tile
 * waiting for a neighbouring tile's values; default 2).  A wait that exceeds
 * it stops all waits of that launch, the launch runs to its end, and the call
 * that issued it (preconditioner apply, solve) returns RSV_ERR_TIMEOUT.  A
 * hang watchdog: the solver's kernels never spin unbounded.
 * Errors: RSV_ERR_ARG (ctx NULL, seconds not in (0, 60]). */
rsv_status rsv_set_wait_limit(rsv_ctx *ctx, double seconds);

/* ---------------------------------------------------------------- grid and MAP */

/* Structured grid nx*ny*nz (Grid section); nx, ny, nz >= 1 and
 * nx*ny*nz*3 < 2^31.  Errors: RSV_ERR_ARG. */
rsv_status rsv_grid_create(rsv_ctx *ctx, int32_t nx, int32_t ny, int32_t nz,
                           int32_t ordering /* rsv_ordering */, rsv_grid **out);
void rsv_grid_destroy(rsv_grid *g);
int64_t rsv_grid_ncell(const rsv_grid *g);
/* Cell -> block row under the grid's ordering (MAP section); the scalar row of
 * component c is 3*block_row + c.  Errors: RSV_ERR_ARG (out of range). */
rsv_status rsv_cell_to_row(const rsv_grid *g, int32_t i, int32_t j, int32_t k, int64_t *block_row);
rsv_status rsv_row_to_cell(const rsv_grid *g, int64_t block_row, int32_t *i, int32_t *j, int32_t *k);

/* ---------------------------------------------------------------- matrix */

/* Assemble the block matrix (Distributed Matrices section) from
 * blocks[ncell][7][3][3] (row-major 3x3), rows in block-row order, slots by
 * direction: 0:-z 1:-y 2:-x 3:diagonal 4:+x 5:+y 6:+z.  `where` says whether
 * `blocks` is a host or a device pointer.  The library copies the values.
 * Errors: RSV_ERR_ARG, RSV_ERR_OOM, RSV_ERR_PATTERN (nonzero block toward a
 * missing neighbour), RSV_ERR_NAN, RSV_ERR_HIP. */
rsv_status rsv_matrix_assemble(rsv_grid *g, const double *blocks, int32_t where, rsv_matrix **out);
/* A scalar system (one unknown per cell, 1x1 blocks: the paper's Poisson
 * Equation example and pressure systems): coef HOST or DEVICE FP64
 * [ncell][7] in block-row order, slots -z,-y,-x,D,+x,+y,+z by cell direction
 * (a coefficient toward a missing neighbour must be 0, else
 * RSV_ERR_PATTERN; non-finite: RSV_ERR_NAN).  Vectors of a scalar matrix
 * have length ncell in block-row order.  rsv_matrix_update, rsv_spmv,
 * rsv_spmv_noalloc (no scratch needed), rsv_precond_setup with RSV_PC_RAS
 * (scalar RAS, FP64) or RSV_PC_BILU0 (ILU(0) of the whole grid: RAS with one
 * subdomain and no overlap) or RSV_PC_NONE, rsv_precond_apply and rsv_solve
 * (GMRES, BiCGSTAB) accept it; the learned preconditioner does not. */
rsv_status rsv_matrix_assemble_scalar(rsv_grid *g, const double *coef, int32_t where, rsv_matrix **out);
/* New values, same grid (next Newton step).  Preconditioners built on the
 * old values must be set up again.  Errors as for assemble. */
rsv_status rsv_matrix_update(rsv_matrix *A, const double *blocks, int32_t where);
void rsv_matrix_destroy(rsv_matrix *A);
/* y = alpha*A*x + beta*y (Algebraic Operations: y = alpha A x + beta y);
 * x, y device vectors of length 3*ncell (must not alias). */
rsv_status rsv_spmv(rsv_matrix *A, double alpha, const double *x, double beta, double *y);
/* The same product for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the tile-lane staging copies of x and A x live in a fixed
 * per-device scratch array of RSV_NOALLOC_SCRATCH_BYTES that the library
 * holds from the first context on the device until the process ends, so no
 * call allocates (rsv_spmv reserves the matrix's solver workspace instead).
 * The grid must satisfy 2 x 3 x (padded cells) x 8 bytes <= the scratch size,
 * i.e. 48 x ceil(nx/8) x ceil(ny/8) x 64 x nz <= RSV_NOALLOC_SCRATCH_BYTES
 * (128x128x64 fits), else RSV_ERR_ARG and nothing runs.  Every call on a
 * device shares that device's scratch: calls that overlap on one GPU (two
 * streams, two host threads) race and must be ordered by the caller.  Each
 * call writes all the scratch it reads, so nothing carries over between
 * calls.  Synchronises the context's stream before returning, like rsv_spmv. */
#define RSV_NOALLOC_SCRATCH_BYTES (64ll << 20)
rsv_status rsv_spmv_noalloc(rsv_matrix *A, double alpha, const double *x, double beta, double *y);
/* y = alpha*x + beta*y on device vectors of length n (the vector update of
 * the Algebraic Operations subsection), enqueued on the context's stream
 * without a synchronisation; x and y may be the same vector.  beta = 0 does
 * not read y.  Used, for example, to form training targets e = x_true - x. */
rsv_status rsv_axpby(rsv_ctx *ctx, int64_t n, double alpha, const double *x, double beta, double *y);
/* Device bytes held by the matrix and its solver workspace (diagnostics;
 * preconditioners are separate objects and not counted). */
int64_t rsv_matrix_device_bytes(const rsv_matrix *A);

/* ---------------------------------------------------------------- preconditioner */

void rsv_pc_params_default(rsv_pc_params *p);
/* Build the preconditioner (SOLVER_PC assemble hook): BILU0 factorisation,
 * RAS subdomains + local factorisations, the learned network plus its
 * BILU0 fallback, or a CPR preconditioner (its stage R, the decoupling
 * weights, A_pp and the multigrid hierarchy with the inverse of its
 * coarsest level).  Errors: RSV_ERR_ARG, RSV_ERR_OOM, RSV_ERR_ZERO_PIVOT
 * (the offending block row is written to *bad_cell if non-NULL), RSV_ERR_HIP. */
rsv_status rsv_precond_setup(rsv_matrix *A, const rsv_pc_params *p, rsv_precond **out, int64_t *bad_cell);
/* z = M^{-1} r (SOLVER_PC solve hook); r, z device vectors, may not alias.
 * For LEARNED this applies the network (no fallback). */
rsv_status rsv_precond_apply(rsv_precond *M, const double *r, double *z);
void rsv_precond_destroy(rsv_precond *M);
/* CPR diagnostics (RSV_PC_CPR only; else RSV_ERR_ARG).
 * rsv_cpr_levels: the multigrid's level count into *nlevels and, for
 *   l < min(nlevels, cap), the grid of level l into dims[3l .. 3l+2] (HOST).
 * rsv_cpr_pressure_matrix: the seven coefficients of every row of level l
 *   (level 0 = A_pp) into the HOST array coef[n_l][7], rows in the order
 *   i + nx (j + ny k') of that level's grid, where k' is the block-row layer
 *   (the layer of the grid's ordering), slots -z,-y,-x,D,+x,+y,+z in k'.
 * rsv_cpr_weights: the decoupling weights w_c into the HOST array w[ncell][3],
 *   block-row order.
 * rsv_cpr_pressure_apply: x = M_g(A_pp)^-1 b, one V-cycle; b and x DEVICE
 *   vectors of length ncell in block-row order (may not alias). */
rsv_status rsv_cpr_levels(const rsv_precond *M, int32_t *nlevels, int32_t *dims, int32_t cap);
rsv_status rsv_cpr_pressure_matrix(const rsv_precond *M, int32_t level, double *coef);
rsv_status rsv_cpr_weights(const rsv_precond *M, double *w);
rsv_status rsv_cpr_pressure_apply(rsv_precond *M, const double *b, double *x);
/* Diagnostics: the block ILU(0) factors of an FP64 BILU0 preconditioner
 * (Preconditioners section, ILU(0) of the block matrix), copied to HOST
 * arrays in block-row order: L[row][3][3][3], the unit-lower blocks
 * L_ck = A_ck D_k^-1 toward the -z, -y, -x neighbours (zero where a
 * neighbour is absent), and Dinv[row][3][3], the inverted pivot blocks.
 * The caller owns both arrays (27 and 9 doubles per cell).  RSV_ERR_ARG for
 * another preconditioner type or the FP32 form. */
rsv_status rsv_precond_bilu0_factors(const rsv_precond *M, double *L, double *Dinv);
/* Diagnostics: the bytes one apply must move at least -- each factor entry,
 * index and vector read or written once -- for the level-scheduled local
 * solvers (ILU(k) with k >= 1, ILUT, the scalar RAS); -1 for the others (their
 * byte counts are stated with their kernels) or a NULL preconditioner. */
int64_t rsv_precond_apply_bytes(const rsv_precond *M);

/* ---------------------------------------------------------------- solver */

void rsv_solver_params_default(rsv_solver_params *p);
/* Solve A x = b (Linear System section).  b: device, length 3*ncell.
 * x: device, in: x0, out: the solution or last iterate.  M may be NULL
 * (no preconditioner).  Returns RSV_OK when the recomputed FP64 relative
 * residual meets tol (or rtol/atol), RSV_NOT_CONVERGED after maxit,
 * RSV_BREAKDOWN, or an error.  `st` may be NULL. */
rsv_status rsv_solve(rsv_matrix *A, rsv_precond *M, const rsv_solver_params *p,
                     const double *b, double *x, rsv_stats *st);
/* Residual estimates per step of the last solve with record_history = 1:
 * hist[0] = initial relative residual, hist[s] after step s.  Writes at most
 * cap values to the HOST array hist; returns how many exist. */
int64_t rsv_solve_history(const rsv_matrix *A, double *hist, int64_t cap);

/* ---------------------------------------------------------------- learned preconditioner */

/* U-Net architecture: 3 levels, channels c0/c1/c2 (default 16/32/64),
 * 3x3x3 kernels, 4 input channels (3 residual components + ln k), 3 outputs. */
typedef struct rsv_net_arch {
    int32_t levels;      /* must be 3 */
    int32_t c0, c1, c2;  /* channels per level */
    int32_t reserved[4];
} rsv_net_arch;

/* Create a network with seeded random weights.  Errors: RSV_ERR_ARG, RSV_ERR_OOM. */
rsv_status rsv_net_create(rsv_ctx *ctx, const rsv_net_arch *arch, uint64_t seed, rsv_net **out);
void rsv_net_destroy(rsv_net *net);
/* Number of parameters and FP32 master copies of them (HOST arrays). */
int64_t rsv_net_num_params(const rsv_net *net);
rsv_status rsv_net_get_params(rsv_net *net, float *host_out, int64_t n);
rsv_status rsv_net_set_params(rsv_net *net, const float *host_in, int64_t n);
rsv_status rsv_net_save(rsv_net *net, const char *path);
rsv_status rsv_net_load(rsv_net *net, const char *path);
/* Inference z = ||r||_rms * N(r / ||r||_rms, lnk) on grid g.  r, z: device
 * FP64 vectors (block-row order); lnk: device FP32 per cell (standardised
 * inside).  Errors: RSV_ERR_ARG (grid dims not multiples of 4).  A network
 * keeps one set of activation buffers, sized for the last grid it ran on:
 * calls on one network (inference, training, applies of preconditioners
 * built on it) must not overlap in time. */
rsv_status rsv_net_forward(rsv_net *net, rsv_grid *g, const double *r, const float *lnk, double *z);
/* One Adam step on a batch of `nb` samples on grid g: inputs r[nb][3*ncell]
 * (device FP64), targets e[nb][3*ncell] (device FP64), lnk[nb][ncell]
 * (device FP32).  Loss = mean_b ||N(r_b/s_b) - e_b/s_b||^2 / ||e_b/s_b||^2
 * with s_b = rms(r_b).  The loss is written to *loss_out (host). */
rsv_status rsv_net_train_step(rsv_net *net, rsv_grid *g, int32_t nb, const double *r, const double *e,
                              const float *lnk, float lr, float *loss_out);
/* Forward + backward without the update: loss and the gradient of every
 * parameter (HOST array of rsv_net_num_params floats).  For gradient checks. */
rsv_status rsv_net_loss_grad(rsv_net *net, rsv_grid *g, int32_t nb, const double *r, const double *e,
                             const float *lnk, float *loss_out, float *grad_out);

/* One 3x3x3 convolution layer of the network (zero padding, stride 1), the
 * building block the network's forward and training passes are made of;
 * exposed so each can be checked on its own.  Voxel v = i + nx*(j + ny*k);
 * tensors are channels-last [v][c].  x: DEVICE BF16 bit patterns [V][cin];
 * w: DEVICE FP32 [27][cin][cout] with tap (dk+1)*9 + (dj+1)*3 + (di+1)
 * (rounded to BF16 inside); b: DEVICE FP32 [cout] or NULL; y: DEVICE FP32
 * [V][cout] = b + sum_tap sum_ci w x(shifted).  cin a multiple of 4 up to
 * 64, cout 16, 32 or 64; otherwise RSV_ERR_ARG.  Synchronous. */
rsv_status rsv_conv3d(rsv_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t cin, int32_t cout,
                      const uint16_t *x, const float *w, const float *b, float *y);
/* Its gradients for an output gradient dy (DEVICE BF16 [V][cout]): dx =
 * the adjoint convolution (DEVICE FP32 [V][cin], needs cin 16/32/64),
 * dw (DEVICE FP32 [27][cin][cout]), db (DEVICE FP32 [cout]); any of the
 * three may be NULL.  Synchronous. */
rsv_status rsv_conv3d_bwd(rsv_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t cin, int32_t cout,
                          const uint16_t *x, const float *w, const uint16_t *dy, float *dx, float *dw, float *db);

/* ---------------------------------------------------------------- kernel timing (diagnostics) */

/* Kernel classes timed with HIP events recorded on the context stream
 * around each launch while profiling is enabled. */
enum {
    RSV_K_SPMV = 0,      /* block SpMV (all fused epilogues) */
    RSV_K_ILU_FWD = 1,   /* BILU0 forward sweep */
    RSV_K_ILU_BWD = 2,   /* BILU0 backward sweep */
    RSV_K_RAS = 3,       /* RAS apply (both sweeps of every subdomain) */
    RSV_K_ORTHO = 4,     /* CGS2 multi-dot / update / normalise kernels */
    RSV_K_VEC = 5,       /* other vector kernels (BiCGSTAB updates, copies, reductions) */
    RSV_K_FACTOR = 6,    /* factorisations */
    RSV_K_NET = 7,       /* U-Net kernels */
    RSV_K_CPR = 8,       /* CPR: residual-restriction products, multigrid, prolongation, combination */
    RSV_K_COUNT = 9
};
/* on = 1 starts (and zeroes) the per-class totals, on = 0 stops recording. */
rsv_status rsv_profile_enable(rsv_ctx *ctx, int32_t on);
/* Classes recorded while profiling is on: bit k set records class k (default
 * all).  Each recorded launch adds two events to the stream, so a caller that
 * times whole solves while profiling records only the classes it needs. */
rsv_status rsv_profile_classes(rsv_ctx *ctx, uint32_t mask);
/* Synchronises the stream and writes per-class total milliseconds and launch
 * counts (HOST arrays of RSV_K_COUNT entries; either may be NULL). */
rsv_status rsv_profile_read(rsv_ctx *ctx, double *ms, int64_t *launches);

/* ---------------------------------------------------------------- Hilbert space-filling-curve partition */
/* Space-filling Partitioning Method section.  Keys: each point of [0,1]^3 is
 * scaled by 2^32 - 1 and truncated to three 32-bit coordinates; level l
 * (l = 0 first) reads bit 31 - l of each coordinate (x weight 4, y 2, z 1)
 * and walks the 24-state machine of the paper's ordering and orientation
 * tables (the table-driven Hilbert order figures), giving one base-8 digit
 * per level, most significant first: a key of 3*levels bits.
 *
 * rsv_hsfc_keys: n points, coords DEVICE [n][3] FP64 in [0,1], levels in
 * [1, 21], keys DEVICE uint64 [n].  A coordinate outside [0,1] or not a
 * number: RSV_ERR_ARG (its key is 0).  Synchronises the stream. */
rsv_status rsv_hsfc_keys(rsv_ctx *ctx, int64_t n, const double *coords, int32_t levels, uint64_t *keys);
/* Keys of the grid's cells, DEVICE uint64 [ncell] in block-row order, from
 * the cell centroids ((i, j, k) + 1/2) / max(nx, ny, nz): the linear map of
 * the grid into [0,1)^3 that keeps cells cubic (step 1 of Algorithm
 * "Space-filling curve method"). */
rsv_status rsv_grid_hsfc_keys(rsv_grid *g, int32_t levels, uint64_t *keys);
/* The equal-count cut of the curve (step 3 of that algorithm): with the n
 * keys (DEVICE, from rsv_*hsfc_keys with the same levels) in increasing
 * order, equal keys by index, the entry of rank r goes to part
 * floor(r * nparts / n); part DEVICE int32 [n].  n <= 2^31.  Allocates its
 * sort buffers (24 n bytes plus histograms) for the call. */
rsv_status rsv_hsfc_partition(rsv_ctx *ctx, int64_t n, const uint64_t *keys, int32_t levels, int32_t nparts,
                              int32_t *part);
/* Partition quality (Partition Quality subsection) of part (DEVICE int32
 * [ncell] in block-row order, values in [0, nparts), nparts <= 16384): per
 * part |G_i|, f_i (faces of its cells, each once), b_i (those shared with
 * another part) and c_i (parts it shares a face with).  q (HOST [5]): load
 * imbalance N_p max|G_i| / sum|G_i|, max b_i/f_i, the global surface index
 * sum b_i / (sum f_i - sum b_i), the average (1/N_p) sum b_i/f_i, max c_i.
 * per_part (HOST [nparts][4], nullable).  A part number out of range:
 * RSV_ERR_ARG. */
rsv_status rsv_partition_quality(rsv_grid *g, const int32_t *part, int32_t nparts, double *q, int64_t *per_part);

#ifdef __cplusplus
}
#endif
#endif /* RSV_H */
