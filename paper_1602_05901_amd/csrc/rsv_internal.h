// Internal declarations of the rsv HIP library (gfx950).  Not part of the ABI.
//
// Internal vector/matrix layout ("tile-lane" layout).
//   The x-y plane is cut into 8x8 tiles (NTX x NTY, grid padded with phantom
//   cells up to multiples of 8).  Within a tile the 64 (i,j) columns map to
//   the 64 lanes of a wavefront, sorted by anti-diagonal d = i + j.  Each
//   tile owns nz "rows"; slot (tile T, row r, lane L) holds the cell
//   (8*tx + i_L, 8*ty + j_L, k) with k = (r - d_L) mod nz.
//   This skewed, wrapped placement puts all cells that a hyperplane wavefront
//   step touches in one tile into one 64-wide row, so the ILU sweeps read and
//   write whole rows (fully coalesced), with no padding: it is a bijection
//   between real+phantom cells and slots.
//   slot      = (T*nz + r)*64 + L
//   vector    : v[(slot>>6)*192 + comp*64 + (slot&63)]     (3 comps per row)
//   matrix A  : A[((slot>>6)*63 + e)*64 + (slot&63)], e = dir*9 + 3*p + q,
//               dir 0:-z 1:-y 2:-x 3:diag 4:+x 5:+y 6:+z
//   Phantom slots hold zero in every vector and zero blocks in every matrix.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "rsv.h"

#define RSV_VERSION 10000

// ------------------------------------------------------------------ lanes
// Lanes sorted by anti-diagonal d = i + j (ties by j).  S(d) = first lane of d.
__host__ __device__ inline int lane_first(int d)
{
    return (d <= 8) ? d * (d + 1) / 2 : 64 - (15 - d) * (16 - d) / 2;
}
__host__ __device__ inline int ij_lane(int i, int j)
{
    const int d = i + j;
    return lane_first(d) + j - (d > 7 ? d - 7 : 0);
}
__host__ __device__ inline void lane_ij(int L, int &i, int &j)
{
    int d = 0;
    while (d < 14 && lane_first(d + 1) <= L) ++d;
    j = (d > 7 ? d - 7 : 0) + (L - lane_first(d));
    i = d - j;
}

struct Geo {
    int32_t nx, ny, nz, ntx, nty, ordering;
    int64_t nslot;   // NT*nz*64
};

__host__ __device__ inline int wrap_nz(int v, int nz)
{
    // v in [-nz-15, 2*nz+15]
    while (v < 0) v += nz;
    while (v >= nz) v -= nz;
    return v;
}

__host__ __device__ inline int64_t slot_of(const Geo &g, int gx, int gy, int k)
{
    const int tx = gx >> 3, ty = gy >> 3, i = gx & 7, j = gy & 7;
    const int r = wrap_nz(k + i + j, g.nz);
    return ((int64_t)(ty * g.ntx + tx) * g.nz + r) * 64 + ij_lane(i, j);
}

// Decode a slot; returns false for phantom slots.
__host__ __device__ inline bool cell_of(const Geo &g, int64_t slot, int &gx, int &gy, int &k)
{
    const int L = (int)(slot & 63);
    const int64_t rowi = slot >> 6;
    const int r = (int)(rowi % g.nz);
    const int T = (int)(rowi / g.nz);
    int i, j;
    lane_ij(L, i, j);
    gx = (T % g.ntx) * 8 + i;
    gy = (T / g.ntx) * 8 + j;
    k = wrap_nz(r - i - j, g.nz);
    return gx < g.nx && gy < g.ny;
}

__host__ __device__ inline int64_t vidx(int64_t slot, int p) { return (slot >> 6) * 192 + p * 64 + (slot & 63); }
__host__ __device__ inline int64_t aidx(int64_t slot, int e) { return ((slot >> 6) * 63 + e) * 64 + (slot & 63); }

// block row of a cell under the ABI ordering
__host__ __device__ inline int64_t row_of(const Geo &g, int gx, int gy, int k)
{
    const int kk = (g.ordering == RSV_TOP_DOWN) ? (g.nz - 1 - k) : k;
    return ((int64_t)kk * g.ny + gy) * g.nx + gx;
}

// neighbour offsets by direction
__host__ __device__ inline void dir_off(int s, int &di, int &dj, int &dk)
{
    di = (s == 2) ? -1 : (s == 4) ? 1 : 0;
    dj = (s == 1) ? -1 : (s == 5) ? 1 : 0;
    dk = (s == 0) ? -1 : (s == 6) ? 1 : 0;
}

// ------------------------------------------------------------------ objects

// Device scalar slots (doubles) used by the Krylov drivers.
enum {
    SC_W0 = 0,       // ||A z||^2 before orthogonalisation
    SC_HN = 1,       // ||w||^2 after CGS2
    SC_RR = 2,       // ||r||^2
    SC_RH = 3,       // rhat . r   (written together with SC_RR)
    SC_RV = 4,       // rhat . v
    SC_SS = 5,       // ||s||^2
    SC_TS = 6,       // t . s
    SC_TT = 7,       // t . t      (written together with SC_TS)
    SC_BB = 8,       // ||b||^2
    SC_MISC = 9,
    SC_H1 = 16,      // 64 slots: first CGS pass coefficients
    SC_H2 = 80,      // 64 slots: second pass
    SC_Y = 144,      // 64 slots: least-squares solution
    SC_DP = 256,     // DCGS2: 2K dots of the combined pass (V_i . V_{K-1}, then V_i . w), then 3 step scalars
    SC_COUNT = 400
};

struct rsv_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    double *h_scal = nullptr;     // pinned, SC_COUNT
    double *h_spec = nullptr;     // pinned, 2 x SC_COUNT: scalars copied without a stream sync
    hipEvent_t spec_ev[2] = {nullptr, nullptr};
    double *d_scal = nullptr;     // device, SC_COUNT
    double *d_partials = nullptr; // device partial sums
    int64_t partials_cap = 0;     // doubles
    uint32_t epoch = 1;           // wavefront face-exchange epoch
    uint64_t wait_ticks = 200000000ull;   // bound on a wavefront wait (100 MHz wall clock; 2 s)
    uint64_t *d_tickets = nullptr;// tile ticket counters (8 counters)
    uint64_t ticket_base[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int32_t *d_flags = nullptr;   // [0] error flags, [1] bad cell (min)
    double *d_scratch = nullptr;  // this device's fixed scratch (rsv_spmv_noalloc), not owned
    int num_cu = 256;
    int lds_max = 65536;               // dynamic LDS bytes a workgroup may use
    int lds_per_cu = 0;
    // kernel timing
    bool prof_on = false;
    uint32_t prof_mask = 0xffffffffu;  // kernel classes recorded
    std::vector<hipEvent_t> prof_ev;   // pairs
    std::vector<int> prof_kind;        // per pair
    int prof_used = 0;                 // events recorded (2 per pair)
    double prof_ms[RSV_K_COUNT] = {0};
    int64_t prof_cnt[RSV_K_COUNT] = {0};
};

// Kernel timing: returns a token for prof_end (or -1 when profiling is off).
int prof_begin(rsv_ctx *c, int kind);
void prof_end(rsv_ctx *c, int tok);
struct ProfScope {
    rsv_ctx *c;
    int tok;
    ProfScope(rsv_ctx *c_, int kind) : c(c_), tok(prof_begin(c_, kind)) {}
    ~ProfScope() { prof_end(c, tok); }
};

struct rsv_grid {
    rsv_ctx *ctx = nullptr;
    Geo geo{};
    int64_t ncell = 0;
    int64_t nv = 0;               // internal vector length (3*nslot)
    int nplanes = 0;              // nx+ny+nz-2 hyperplanes
    std::vector<int64_t> plane_ptr;   // host, nplanes+1
    int32_t *d_plane_slots = nullptr; // device, real slots sorted by (plane, slot)
};

struct SolverWork;

struct rsv_matrix {
    rsv_grid *g = nullptr;
    int bs = 3;                       // unknowns per cell: 3 (block matrices) or 1 (scalar)
    int64_t nv = 0;                   // solver vector length: tile-lane 3*nslot, or ncell in row order
    double *d_A = nullptr;            // bs 3: tile-lane blocks, nslot/64 * 63 * 64 doubles
    double *d_coef = nullptr;         // bs 1: coef[slot][row], 7 * ncell doubles
    SolverWork *ws = nullptr;
    std::vector<double> hist;
    int64_t bytes = 0;
};

struct PcImpl {
    virtual ~PcImpl() {}
    // z = M^{-1} r on tile-lane vectors (length nv); no aliasing
    virtual rsv_status apply(const double *r_tl, double *z_tl) = 0;
    virtual int64_t bytes() const = 0;
    // algorithmic bytes one apply moves (factor data read once, vectors); -1: not stated
    virtual int64_t apply_bytes() const { return -1; }
    // FP64 BILU0 only: the factors in block-row order into host arrays
    virtual rsv_status bilu0_factors(double * /*L*/, double * /*Dinv*/) { return RSV_ERR_ARG; }
};

struct rsv_precond {
    rsv_matrix *A = nullptr;
    rsv_pc_params p{};
    PcImpl *impl = nullptr;       // BILU0 / RAS / learned
    PcImpl *fallback = nullptr;   // BILU0 for LEARNED
};

// ------------------------------------------------------------------ error helpers
rsv_status set_err(rsv_ctx *c, rsv_status s, const std::string &msg);
#define RSV_HIP(ctx, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return set_err((ctx), RSV_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
#define RSV_LAUNCH(ctx)                                                                      \
    do {                                                                                     \
        hipError_t e_ = hipGetLastError();                                                   \
        if (e_ != hipSuccess)                                                                \
            return set_err((ctx), RSV_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

// allocation helpers (record size)
rsv_status dev_alloc(rsv_ctx *c, void **p, size_t bytes);
void dev_free(void *p);

// ------------------------------------------------------------------ launchers (rsv_kernels.hip)
// Each returns RSV_OK or RSV_ERR_HIP on launch failure.
rsv_status partials_reserve(rsv_ctx *c, int64_t ndoubles);
int spmv_blocks(const Geo &g);
int vec_blocks(int64_t n);

enum SpmvMode { SPMV_Y = 0, SPMV_AXPBY = 1, SPMV_RESID = 2, SPMV_NORM = 3, SPMV_DOT1 = 4, SPMV_DOT2 = 5 };
// SPMV_Y: y = A x.  SPMV_AXPBY: y = alpha A x + beta y.  SPMV_RESID: y = b - A x, partial ||y||^2 -> sc[k0].
// SPMV_NORM: y = A x, ||y||^2 -> sc[k0].  SPMV_DOT1: y = A x, aux1.y -> sc[k0].
// SPMV_DOT2: y = A x, y.aux1 -> sc[k0], y.y -> sc[k0+1].
rsv_status launch_spmv(rsv_ctx *c, const Geo &g, const double *A, int mode, const double *x, double *y,
                       const double *aux1, double alpha, double beta, int k0);

rsv_status launch_reduce(rsv_ctx *c, int nblocks, int K, int k0);    // partials[nblocks][K] -> d_scal[k0..]

// scalar systems (rsv_scalar.hip): the product with the same modes, and the
// matrix-independent front ends the Krylov drivers use
rsv_status launch_sspmv(rsv_ctx *c, const Geo &g, const double *coef, int mode, const double *x, double *y,
                        const double *aux, double alpha, double beta, int k0);
rsv_status mat_spmv(rsv_matrix *M, int mode, const double *x, double *y, const double *aux, double alpha,
                    double beta, int k0);
rsv_status mat_in(rsv_matrix *M, const double *nat, double *v);                       // ABI order -> solver layout
rsv_status mat_out(rsv_matrix *M, const double *v, double *nat, double alpha, double beta);   // nat = a v + b nat
rsv_status scalar_assemble_values(rsv_matrix *M, const double *coef, int32_t where);
rsv_status sras_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell);
// ILU(k), k >= 1, for 3x3-block matrices (rsv_iluk.hip): RAS local solvers, or the whole grid as one subdomain
rsv_status rasK_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell);
// ILUT(p, tol) for 3x3-block matrices (rsv_iluk.hip): RAS local solvers, or the whole grid
rsv_status rasT_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell);

rsv_status launch_nat_to_tl(rsv_ctx *c, const Geo &g, const double *nat, double *tl);
rsv_status launch_tl_to_nat(rsv_ctx *c, const Geo &g, const double *tl, double *nat, double alpha, double beta);
rsv_status launch_assemble(rsv_ctx *c, const Geo &g, const double *blocks_nat_dev, double *A);

// vector ops on length-n arrays
rsv_status launch_dot(rsv_ctx *c, int64_t n, const double *x, const double *y, int k0);   // x.y -> sc[k0]
rsv_status launch_copy(rsv_ctx *c, int64_t n, const double *x, double *y);
rsv_status launch_scale_dev(rsv_ctx *c, int64_t n, double *x, int k_norm2);   // x /= sqrt(sc[k]) (0 -> 0)
rsv_status launch_axpby(rsv_ctx *c, int64_t n, double a, const double *x, double b, double *y); // y = a x + b y
rsv_status launch_mdot(rsv_ctx *c, int64_t n, const double *V, int64_t ldv, int K, const double *w, int k0);
// CGS2's second pass: dots of V_i with w - V c (c = scalars kc..), w unchanged
rsv_status launch_upd_dot(rsv_ctx *c, int64_t n, const double *V, int64_t ldv, int K, double *w, int kc, int k0);
// CGS2's third pass: w <- (w - V c1) - V c2 (scalars kc1.., kc2..) and w . w
rsv_status launch_upd_norm(rsv_ctx *c, int64_t n, const double *V, int64_t ldv, int K, double *w, int kc1, int kc2,
                           int k0);
rsv_status launch_combine(rsv_ctx *c, int64_t n, const double *V, int64_t ldv, int K, int ky, double *u, int accumulate);
// Fixed per-device scratch of the entry points that allocate nothing
// (RSV_NOALLOC_SCRATCH_BYTES in rsv.h), in doubles.
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = (int64_t)RSV_NOALLOC_SCRATCH_BYTES / 8;
constexpr int MAX_DEVICES = 64;
rsv_status scratch_lookup(rsv_ctx *c);

// DCGS2 step with K = j + 1 basis vectors V_0..V_j and w = V_{j+1}: the dots
// V_i . [V_j, w] into d_scal[k0 .. k0 + 2K), then the combined update (V_j
// corrected, w projected and normalised; four step scalars after the dots)
// DCGS2 breakdown threshold: a squared norm below this fraction of ||w||^2,
// obtained as a difference of squares, is lost to rounding
constexpr double DCGS_LOST = 64.0 * 2.220446049250313e-16;   // 64 x DBL_EPSILON
rsv_status launch_dcgs_dots(rsv_ctx *c, int64_t n, const double *V, int64_t ldv, int K, const double *w, int k0);
rsv_status launch_dcgs_update(rsv_ctx *c, int64_t n, double *V, int64_t ldv, int K, double *w, int kd);
// BiCGSTAB fused vector updates
rsv_status launch_bicg_p(rsv_ctx *c, int64_t n, const double *r, const double *v, double beta, double omega, double *p);
rsv_status launch_bicg_s(rsv_ctx *c, int64_t n, const double *r, const double *v, double *s, int k_alpha_num, int k_alpha_den, int k0);
rsv_status launch_bicg_xr(rsv_ctx *c, int64_t n, double alpha, double omega, const double *ph, const double *sh,
                          const double *s, const double *t, const double *rh, double *x, double *r, int k0);
rsv_status launch_nonfinite(rsv_ctx *c, int64_t n, const double *x, int k0);   // count of non-finite -> sc[k0]

// scalars
rsv_status scal_to_host(rsv_ctx *c, int k0, int n);   // sync copy d_scal[k0..k0+n) -> h_scal
// async copy d_scal[k0..k0+n) -> h_spec[buf][k0..] and an event after it; scal_wait blocks on that event
rsv_status scal_to_host_async(rsv_ctx *c, int buf, int k0, int n);
rsv_status scal_wait(rsv_ctx *c, int buf);
rsv_status scal_set(rsv_ctx *c, int k0, const double *vals, int n);

// A grid whose factorisation "hyperplanes" are (i mod mx) + (j mod my) + (k mod mz):
// for a grid of independent boxes of mx x my x mz cells (rsv_grid_create: the
// plain hyperplanes, mx = nx, my = ny, mz = nz).
rsv_status grid_create_planes(rsv_ctx *c, int32_t nx, int32_t ny, int32_t nz, int32_t ordering, int mx, int my,
                              int mz, rsv_grid **out);

// ------------------------------------------------------------------ preconditioners
rsv_status bilu0_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell);
// BILU0 of a grid made of independent boxes of btx x bty tiles (all couplings
// between boxes zero): the pipelined sweeps exchange faces only inside a box.
// zmap (optional, device, [nslot], not owned): the apply writes the result of
// slot s to slot zmap[s] of its output (nothing when -1) instead of slot s.
rsv_status bilu0_create_boxed(rsv_matrix *A, const rsv_pc_params *p, int btx, int bty, const int32_t *zmap,
                              PcImpl **out, int64_t *bad_cell);
rsv_status ras_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell);
// CPR-type two-stage preconditioner around the stage R (owned by the result,
// deleted on failure); p carries the variant, decoupling and multigrid fields
rsv_status cpr_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl *stage, PcImpl **out, int64_t *bad_cell);
// base: the BILU0 preconditioner a learned_mode 1 network corrects (not owned)
rsv_status learned_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, PcImpl *base);
// LDS ring depth (slots) of the pipelined BILU0 sweeps for this device
int64_t sweep_ring_depth(const rsv_ctx *c, int dir, int fp32);

// pinned host error flag read (after sync); flags: bit0 timeout, bit1 zero pivot, bit2 pattern, bit3 nan
rsv_status flags_check(rsv_ctx *c, int64_t *bad_cell);
rsv_status flags_reset(rsv_ctx *c);
enum { FLAG_TIMEOUT = 1, FLAG_PIVOT = 2, FLAG_PATTERN = 4, FLAG_NAN = 8 };

// 3x3 inverse by cofactors (adjugate / determinant).  Returns false when the
// block is numerically singular: |det| <= 1e-300 or 1-norm condition > 1e14.
__host__ __device__ inline bool inv3(const double *a, double *o)
{
    const double c00 = a[4] * a[8] - a[5] * a[7];
    const double c01 = a[5] * a[6] - a[3] * a[8];
    const double c02 = a[3] * a[7] - a[4] * a[6];
    const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    if (!(fabs(det) > 1e-300)) return false;
    const double id = 1.0 / det;
    o[0] = c00 * id;
    o[1] = (a[2] * a[7] - a[1] * a[8]) * id;
    o[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    o[3] = c01 * id;
    o[4] = (a[0] * a[8] - a[2] * a[6]) * id;
    o[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    o[6] = c02 * id;
    o[7] = (a[1] * a[6] - a[0] * a[7]) * id;
    o[8] = (a[0] * a[4] - a[1] * a[3]) * id;
    double na = 0.0, ni = 0.0;
    for (int q = 0; q < 3; ++q) {
        const double sa = fabs(a[q]) + fabs(a[3 + q]) + fabs(a[6 + q]);
        const double si = fabs(o[q]) + fabs(o[3 + q]) + fabs(o[6 + q]);
        na = sa > na ? sa : na;
        ni = si > ni ? si : ni;
    }
    return na * ni <= 1e14;
}
