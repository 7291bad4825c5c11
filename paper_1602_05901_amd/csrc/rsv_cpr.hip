// CPR-type two-stage preconditioners for the 3x3-block systems (CPR-like
// Preconditioners subsection: the CPR-FP, CPR-PF, CPR-FPF and CPR-FFPF
// algorithms), with a structured aggregation multigrid in place of the
// library AMG the paper uses for the pressure solve M_g(A_pp)^-1.
//
// Stage R: any block preconditioner of this library (RAS, BILU0; FP64 or
// FP32 sweeps), applied on tile-lane vectors.
//
// Pressure stage: the decoupling weights w_c (one 3-vector per cell, from the
// diagonal block) and A_pp(c, n) = w_c^T A_cn e_0 are formed once by one
// thread per tile-lane slot.  The pressure hierarchy lives in plain row order
// of the block rows (i + nx (j + ny k'), k' the layer of the grid's
// numbering): level l holds coef[s][row] (slots -z,-y,-x,D,+x,+y,+z in k'),
// b and x.  Level l+1 aggregates 2x2x2 cells of level l; its Galerkin
// operator P^T A P is again a 7-point stencil (aggregates are boxes, so a
// coupling between two aggregates is a coupling between face neighbours),
// summed by one thread per coarse cell over its fine cells in ascending
// order.  Smoothing is red-black Gauss-Seidel, one launch per colour, one
// thread per cell of that colour.  The coarsest level (at most mg_coarse
// cells) is inverted once by Gauss-Jordan elimination with partial pivoting
// in one workgroup; its solve is a product with the stored inverse.
//
// Fusions: the residual that feeds the pressure stage is formed and
// restricted in one pass (q = w . (f - A x) per slot, r itself is never
// stored); the prolongation x_p += e is folded into the next residual
// product (it reads x + Pi_p e) and into the final combination
// z = (z + Pi_p e) + t; the first pre-smoothing sweep starts from zero
// without reading x; the prolongation of the coarse correction is folded
// into the first post-smoothing sweep (black then red: the black sweep reads
// its red neighbours plus their aggregates' corrections, and every value
// without the correction is overwritten before anything reads it).
#include "rsv_internal.h"

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

namespace {

constexpr int CB = 256;            // threads per block of the per-cell kernels
constexpr int GJ_T = 1024;         // threads of the coarsest level's workgroup
constexpr int MG_MAX_LEVELS = 40;

__device__ __host__ inline int cdim(int v) { return v > 1 ? (v + 1) / 2 : 1; }

// decoupling weights of one cell from its diagonal block d (row-major)
__device__ inline bool cpr_weights(const double *d, int decouple, double *w)
{
    if (decouple == RSV_DECOUPLE_QUASI_IMPES) {
        // w1 d[1][q] + w2 d[2][q] = -d[0][q], q = 1, 2
        const double det = d[4] * d[8] - d[7] * d[5];
        const double scale = fabs(d[4] * d[8]) + fabs(d[7] * d[5]);
        if (!(fabs(det) > 1e-14 * scale) || !(fabs(det) > 1e-300)) return false;
        w[0] = 1.0;
        w[1] = (-d[1] * d[8] + d[7] * d[2]) / det;
        w[2] = (-d[4] * d[2] + d[1] * d[5]) / det;
        return true;
    }
    if (decouple == RSV_DECOUPLE_ABF) {
        double inv[9];
        if (!inv3(d, inv)) return false;
        w[0] = inv[0];
        w[1] = inv[1];
        w[2] = inv[2];
        return true;
    }
    w[0] = 1.0;
    w[1] = 0.0;
    w[2] = 0.0;
    return true;
}

// slot of the block-row numbering's stencil for a direction of the grid
__device__ inline int row_dir(const Geo &g, int s)
{
    return (g.ordering == RSV_TOP_DOWN && (s == 0 || s == 6)) ? 6 - s : s;
}

__global__ __launch_bounds__(CB) void k_cpr_extract(Geo g, const double *__restrict__ A, int decouple,
                                                    double *__restrict__ w, double *__restrict__ coef,
                                                    int32_t *flags)
{
    const int64_t slot = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (slot >= g.nslot) return;
    int gx, gy, k;
    if (!cell_of(g, slot, gx, gy, k)) {
        for (int p = 0; p < 3; ++p) w[vidx(slot, p)] = 0.0;
        return;
    }
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t row = row_of(g, gx, gy, k);
    double d[9], wv[3];
    for (int e = 0; e < 9; ++e) d[e] = A[aidx(slot, 27 + e)];
    if (!cpr_weights(d, decouple, wv)) {
        atomicOr(&flags[0], (int32_t)FLAG_PIVOT);
        atomicMin(&flags[1], (int32_t)row);
        wv[0] = wv[1] = wv[2] = 0.0;
    }
    for (int p = 0; p < 3; ++p) w[vidx(slot, p)] = wv[p];
    for (int s = 0; s < 7; ++s) {
        const double v = wv[0] * A[aidx(slot, s * 9 + 0)] + wv[1] * A[aidx(slot, s * 9 + 3)] +
                         wv[2] * A[aidx(slot, s * 9 + 6)];
        coef[(int64_t)row_dir(g, s) * n + row] = v;
    }
}

// Residual of the block system at x + Pi_p e (x NULL: zero; e NULL: none,
// e in row order).  MODE 0: q[row] = w . (f - A (x + Pi_p e)), the restricted
// residual (r not stored).  MODE 1: r = f - A (x + Pi_p e).
template <int MODE, typename T>
__global__ __launch_bounds__(CB) void k_cpr_resid(Geo g, const T *__restrict__ A, const double *__restrict__ x,
                                                  const double *__restrict__ e, const double *__restrict__ f,
                                                  double *__restrict__ r, const double *__restrict__ w,
                                                  double *__restrict__ q)
{
    const int64_t slot = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (slot >= g.nslot) return;
    int gx = 0, gy = 0, k = 0;
    const bool real = cell_of(g, slot, gx, gy, k);
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    if (real) {
#pragma unroll
        for (int s = 0; s < 7; ++s) {
            int di, dj, dk;
            dir_off(s, di, dj, dk);
            const int ax = gx + di, ay = gy + dj, az = k + dk;
            double x0 = 0.0, x1 = 0.0, x2 = 0.0;
            if (ax >= 0 && ax < g.nx && ay >= 0 && ay < g.ny && az >= 0 && az < g.nz) {
                const int64_t ns = (s == 3) ? slot : slot_of(g, ax, ay, az);
                if (x) {
                    x0 = x[vidx(ns, 0)];
                    x1 = x[vidx(ns, 1)];
                    x2 = x[vidx(ns, 2)];
                }
                if (e) x0 += e[row_of(g, ax, ay, az)];
            }
            const T *a = A + aidx(slot, s * 9);
            acc0 += (double)a[0 * 64] * x0 + (double)a[1 * 64] * x1 + (double)a[2 * 64] * x2;
            acc1 += (double)a[3 * 64] * x0 + (double)a[4 * 64] * x1 + (double)a[5 * 64] * x2;
            acc2 += (double)a[6 * 64] * x0 + (double)a[7 * 64] * x1 + (double)a[8 * 64] * x2;
        }
    }
    const int64_t i0 = vidx(slot, 0), i1 = vidx(slot, 1), i2 = vidx(slot, 2);
    const double r0 = f[i0] - acc0, r1 = f[i1] - acc1, r2 = f[i2] - acc2;
    if (MODE == 0) {
        if (real) q[row_of(g, gx, gy, k)] = w[i0] * r0 + w[i1] * r1 + w[i2] * r2;
    } else {
        r[i0] = r0;
        r[i1] = r1;
        r[i2] = r2;
    }
}

// q[row] = w . f
__global__ __launch_bounds__(CB) void k_cpr_restrict(Geo g, const double *__restrict__ w,
                                                     const double *__restrict__ f, double *__restrict__ q)
{
    const int64_t slot = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (slot >= g.nslot) return;
    int gx, gy, k;
    if (!cell_of(g, slot, gx, gy, k)) return;
    const int64_t i0 = vidx(slot, 0), i1 = vidx(slot, 1), i2 = vidx(slot, 2);
    q[row_of(g, gx, gy, k)] = w[i0] * f[i0] + w[i1] * f[i1] + w[i2] * f[i2];
}

// z = (z + Pi_p e) + t, or z = Pi_p e + t when has_z = 0; e NULL: z (+)= t
__global__ __launch_bounds__(CB) void k_cpr_combine(Geo g, double *__restrict__ z, const double *__restrict__ e,
                                                    const double *__restrict__ t, int has_z)
{
    const int64_t slot = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (slot >= g.nslot) return;
    int gx, gy, k;
    const bool real = cell_of(g, slot, gx, gy, k);
    const int64_t i0 = vidx(slot, 0), i1 = vidx(slot, 1), i2 = vidx(slot, 2);
    double z0 = has_z ? z[i0] : 0.0, z1 = has_z ? z[i1] : 0.0, z2 = has_z ? z[i2] : 0.0;
    if (real && e) z0 += e[row_of(g, gx, gy, k)];
    z[i0] = z0 + t[i0];
    z[i1] = z1 + t[i1];
    z[i2] = z2 + t[i2];
}

// z_p += e
__global__ __launch_bounds__(CB) void k_cpr_prolong(Geo g, double *__restrict__ z, const double *__restrict__ e)
{
    const int64_t slot = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (slot >= g.nslot) return;
    int gx, gy, k;
    if (!cell_of(g, slot, gx, gy, k)) return;
    z[vidx(slot, 0)] += e[row_of(g, gx, gy, k)];
}

// ---------------------------------------------------------------- multigrid

struct LevelGeo {
    int nx, ny, nz;
};

__device__ inline int64_t lidx(const LevelGeo &L, int i, int j, int k)
{
    return ((int64_t)k * L.ny + j) * L.nx + i;
}

__device__ inline int64_t agg_of(const LevelGeo &F, const LevelGeo &C, int i, int j, int k)
{
    return lidx(C, F.nx > 1 ? i >> 1 : 0, F.ny > 1 ? j >> 1 : 0, F.nz > 1 ? k >> 1 : 0);
}

// One Gauss-Seidel sweep over the cells of one colour ((i + j + k) & 1 ==
// colour), one thread per such cell.  zero: x = 0 on entry (no reads of x);
// xc (nullable): read every neighbour as x + xc[aggregate of the neighbour]
// (the coarse correction not yet added to x).
template <typename T>
__global__ __launch_bounds__(CB) void k_mg_gs(LevelGeo L, const T *__restrict__ coef,
                                              const double *__restrict__ b, double *__restrict__ x, int colour,
                                              int zero, const double *__restrict__ xc, LevelGeo C)
{
    const int hx = (L.nx + 1) >> 1;
    const int64_t t = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (t >= (int64_t)hx * L.ny * L.nz) return;
    const int m = (int)(t % hx);
    const int64_t yz = t / hx;
    const int j = (int)(yz % L.ny), k = (int)(yz / L.ny);
    const int i = 2 * m + ((colour + j + k) & 1);
    if (i >= L.nx) return;
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    const int64_t c = lidx(L, i, j, k);
    double s = b[c];
    if (!zero) {
#pragma unroll
        for (int d = 0; d < 7; ++d) {
            if (d == 3) continue;
            int di, dj, dk;
            dir_off(d, di, dj, dk);
            const int a = i + di, bb = j + dj, cc = k + dk;
            if (a < 0 || a >= L.nx || bb < 0 || bb >= L.ny || cc < 0 || cc >= L.nz) continue;
            double v = x[lidx(L, a, bb, cc)];
            if (xc) v += xc[agg_of(L, C, a, bb, cc)];
            s -= (double)coef[d * n + c] * v;
        }
    }
    x[c] = s / (double)coef[3 * n + c];
}

// bc[I] = sum over the fine cells of aggregate I (ascending) of (b - A x)
template <typename T>
__global__ __launch_bounds__(CB) void k_mg_restrict(LevelGeo F, const T *__restrict__ coef,
                                                    const double *__restrict__ b, const double *__restrict__ x,
                                                    LevelGeo C, double *__restrict__ bc)
{
    const int64_t I = (int64_t)blockIdx.x * CB + threadIdx.x;
    const int64_t nc = (int64_t)C.nx * C.ny * C.nz;
    if (I >= nc) return;
    const int ci = (int)(I % C.nx), cj = (int)((I / C.nx) % C.ny), ck = (int)(I / ((int64_t)C.nx * C.ny));
    const int i0 = F.nx > 1 ? 2 * ci : 0, i1 = F.nx > 1 ? min(2 * ci + 2, F.nx) : 1;
    const int j0 = F.ny > 1 ? 2 * cj : 0, j1 = F.ny > 1 ? min(2 * cj + 2, F.ny) : 1;
    const int k0 = F.nz > 1 ? 2 * ck : 0, k1 = F.nz > 1 ? min(2 * ck + 2, F.nz) : 1;
    const int64_t n = (int64_t)F.nx * F.ny * F.nz;
    double sum = 0.0;
    for (int k = k0; k < k1; ++k)
        for (int j = j0; j < j1; ++j)
            for (int i = i0; i < i1; ++i) {
                const int64_t c = lidx(F, i, j, k);
                double ax = 0.0;
#pragma unroll
                for (int d = 0; d < 7; ++d) {
                    int di, dj, dk;
                    dir_off(d, di, dj, dk);
                    const int a = i + di, bb = j + dj, cc = k + dk;
                    if (a < 0 || a >= F.nx || bb < 0 || bb >= F.ny || cc < 0 || cc >= F.nz) continue;
                    ax += (double)coef[d * n + c] * x[lidx(F, a, bb, cc)];
                }
                sum += b[c] - ax;
            }
    bc[I] = sum;
}

// Galerkin coarse operator: one thread per coarse cell, its fine cells in
// ascending order, their couplings in ascending column (slot) order
__global__ __launch_bounds__(CB) void k_mg_galerkin(LevelGeo F, const double *__restrict__ cf, LevelGeo C,
                                                    double *__restrict__ cc_out)
{
    const int64_t I = (int64_t)blockIdx.x * CB + threadIdx.x;
    const int64_t nc = (int64_t)C.nx * C.ny * C.nz;
    if (I >= nc) return;
    const int ci = (int)(I % C.nx), cj = (int)((I / C.nx) % C.ny), ck = (int)(I / ((int64_t)C.nx * C.ny));
    const int i0 = F.nx > 1 ? 2 * ci : 0, i1 = F.nx > 1 ? min(2 * ci + 2, F.nx) : 1;
    const int j0 = F.ny > 1 ? 2 * cj : 0, j1 = F.ny > 1 ? min(2 * cj + 2, F.ny) : 1;
    const int k0 = F.nz > 1 ? 2 * ck : 0, k1 = F.nz > 1 ? min(2 * ck + 2, F.nz) : 1;
    const int64_t n = (int64_t)F.nx * F.ny * F.nz;
    double out[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = k0; k < k1; ++k)
        for (int j = j0; j < j1; ++j)
            for (int i = i0; i < i1; ++i) {
                const int64_t c = lidx(F, i, j, k);
#pragma unroll
                for (int d = 0; d < 7; ++d) {
                    int di, dj, dk;
                    dir_off(d, di, dj, dk);
                    const int a = i + di, bb = j + dj, cc = k + dk;
                    if (a < 0 || a >= F.nx || bb < 0 || bb >= F.ny || cc < 0 || cc >= F.nz) continue;
                    const double v = cf[d * n + c];
                    if (agg_of(F, C, a, bb, cc) == I) out[3] += v;
                    else out[d] += v;
                }
            }
    for (int d = 0; d < 7; ++d) cc_out[d * nc + I] = out[d];
}

// zero diagonal or non-finite coefficient on a level -> zero-pivot flag
// (bad cell: the row on level 0, else none)
__global__ __launch_bounds__(CB) void k_mg_check(int64_t n, const double *__restrict__ coef, int level,
                                                 int32_t *flags)
{
    const int64_t c = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (c >= n) return;
    bool bad = !(coef[3 * n + c] != 0.0);
    for (int d = 0; d < 7; ++d) bad |= !isfinite(coef[d * n + c]);
    if (bad) {
        atomicOr(&flags[0], (int32_t)FLAG_PIVOT);
        if (level == 0) atomicMin(&flags[1], (int32_t)c);
    }
}

// [A | I] of the coarsest level, row-major n x 2n
__global__ __launch_bounds__(CB) void k_mg_dense(LevelGeo L, const double *__restrict__ coef, double *__restrict__ M)
{
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    const int64_t r = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (r >= n) return;
    double *row = M + r * 2 * n;
    for (int64_t q = 0; q < 2 * n; ++q) row[q] = 0.0;
    const int i = (int)(r % L.nx), j = (int)((r / L.nx) % L.ny), k = (int)(r / ((int64_t)L.nx * L.ny));
    for (int d = 0; d < 7; ++d) {
        int di, dj, dk;
        dir_off(d, di, dj, dk);
        const int a = i + di, bb = j + dj, cc = k + dk;
        if (a < 0 || a >= L.nx || bb < 0 || bb >= L.ny || cc < 0 || cc >= L.nz) continue;
        row[lidx(L, a, bb, cc)] = coef[d * n + r];
    }
    row[n + r] = 1.0;
}

// Gauss-Jordan elimination with partial pivoting of [A | I] in one
// workgroup; writes inv (row-major) or raises the zero-pivot flag.
// n <= GJ_T.  After column c is eliminated, the left block's columns < c are
// unit columns and the pivot row is zero there, so each step updates only
// columns >= col; the pivot row is staged in LDS.
__global__ __launch_bounds__(GJ_T) void k_mg_gauss_jordan(int n, double *__restrict__ M, double *__restrict__ inv,
                                                          int32_t *flags)
{
    __shared__ double fac[GJ_T];
    __shared__ double prow[2 * GJ_T];
    __shared__ double red_v[GJ_T / 64];
    __shared__ int red_i[GJ_T / 64];
    __shared__ int piv_s;
    __shared__ double pv_s;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int w2 = 2 * n;
    for (int col = 0; col < n; ++col) {
        // pivot: largest |M[r][col]|, r >= col, first such row on ties
        double bv = -1.0;
        int bi = n;
        for (int r = col + t; r < n; r += GJ_T) {
            const double v = fabs(M[(int64_t)r * w2 + col]);
            if (v > bv) { bv = v; bi = r; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { red_v[wv] = bv; red_i[wv] = bi; }
        __syncthreads();
        if (t == 0) {
            double v = red_v[0];
            int ii = red_i[0];
            for (int q = 1; q < GJ_T / 64; ++q)
                if (red_v[q] > v || (red_v[q] == v && red_i[q] < ii)) { v = red_v[q]; ii = red_i[q]; }
            piv_s = (v > 1e-300 && ii < n) ? ii : -1;
            pv_s = (piv_s >= 0) ? M[(int64_t)piv_s * w2 + col] : 0.0;
        }
        __syncthreads();
        const int piv = piv_s;
        if (piv < 0) {
            if (t == 0) atomicOr(&flags[0], (int32_t)FLAG_PIVOT);
            return;
        }
        // swap rows col and piv, normalise the pivot row into LDS and back
        const double pv = pv_s;
        for (int q = col + t; q < w2; q += GJ_T) {
            const double a = M[(int64_t)col * w2 + q];
            const double p = M[(int64_t)piv * w2 + q];
            if (piv != col) M[(int64_t)piv * w2 + q] = a;
            const double pn = p / pv;
            prow[q] = pn;
            M[(int64_t)col * w2 + q] = pn;
        }
        __syncthreads();
        for (int r = t; r < n; r += GJ_T) fac[r] = (r == col) ? 0.0 : M[(int64_t)r * w2 + col];
        __syncthreads();
        // one wavefront per row, its lanes along the row, four loads in flight
        for (int r = wv; r < n; r += GJ_T / 64) {
            if (r == col) continue;
            const double fr = fac[r];
            double *row = M + (int64_t)r * w2;
            int q = col + lane;
            for (; q + 192 < w2; q += 256) {
                const double a0 = row[q], a1 = row[q + 64], a2 = row[q + 128], a3 = row[q + 192];
                row[q] = a0 - fr * prow[q];
                row[q + 64] = a1 - fr * prow[q + 64];
                row[q + 128] = a2 - fr * prow[q + 128];
                row[q + 192] = a3 - fr * prow[q + 192];
            }
            for (; q < w2; q += 64) row[q] -= fr * prow[q];
        }
        __syncthreads();
    }
    for (int64_t idx = t; idx < (int64_t)n * n; idx += GJ_T) {
        const int r = (int)(idx / n), q = (int)(idx - (int64_t)r * n);
        inv[idx] = M[(int64_t)r * w2 + n + q];
    }
}

// x = inv b on the coarsest level: 16 rows per workgroup, 16 lanes per row
// along it (coalesced row segments), lanes combined by shuffles
constexpr int CO_ROWS = 16;
__global__ __launch_bounds__(CB) void k_mg_coarse(int n, const double *__restrict__ inv,
                                                  const double *__restrict__ b, double *__restrict__ x)
{
    const int l = threadIdx.x & 15;
    const int r = blockIdx.x * CO_ROWS + (threadIdx.x >> 4);
    double acc = 0.0;
    if (r < n) {
        const double *row = inv + (int64_t)r * n;
        for (int q = l; q < n; q += 16) acc += row[q] * b[q];
    }
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    if (r < n && l == 0) x[r] = acc;
}

inline int nblk(int64_t n) { return (int)((n + CB - 1) / CB); }

// FP64 -> FP32 copy
__global__ __launch_bounds__(CB) void k_to_f32(int64_t n, const double *__restrict__ in, float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

struct MgLevel {
    LevelGeo geo{1, 1, 1};
    int64_t n = 0;
    double *coef = nullptr, *b = nullptr, *x = nullptr;
    float *coef32 = nullptr;      // FP32 form: the coefficients the cycle reads
};

struct CprImpl : PcImpl {
    rsv_matrix *A = nullptr;
    rsv_ctx *c = nullptr;
    PcImpl *R = nullptr;          // owned
    int variant = RSV_CPR_FPF, pre = 1, post = 1;
    double *w = nullptr;          // tile-lane, 3 per slot
    double *r = nullptr, *t = nullptr;   // tile-lane work vectors
    double *inv = nullptr;        // coarsest inverse, row-major
    float *A32 = nullptr;         // FP32 form: tile-lane FP32 copy of A for the residual products
    bool fp32 = false;
    std::vector<MgLevel> lev;
    int64_t nbytes = 0;

    ~CprImpl() override
    {
        delete R;
        dev_free(w);
        dev_free(r);
        dev_free(t);
        dev_free(inv);
        dev_free(A32);
        for (auto &L : lev) {
            dev_free(L.coef32);
            dev_free(L.coef);
            dev_free(L.b);
            dev_free(L.x);
        }
    }
    int64_t bytes() const override { return nbytes + (R ? R->bytes() : 0); }

    rsv_status alloc(double **p, int64_t ndoubles)
    {
        nbytes += ndoubles * 8;
        return dev_alloc(c, (void **)p, (size_t)ndoubles * 8);
    }

    rsv_status cycle(int l) { return fp32 ? cycle_t<float>(l) : cycle_t<double>(l); }

    template <typename T>
    static const T *coef_of(const MgLevel &L);

    template <typename T>
    rsv_status cycle_t(int l)
    {
        MgLevel &L = lev[l];
        const T *cf = coef_of<T>(L);
        if (l == (int)lev.size() - 1) {
            hipLaunchKernelGGL(k_mg_coarse, dim3((int)((L.n + CO_ROWS - 1) / CO_ROWS)), dim3(CB), 0, c->stream,
                               (int)L.n, (const double *)inv, L.b, L.x);
            RSV_LAUNCH(c);
            return RSV_OK;
        }
        MgLevel &C = lev[l + 1];
        const int64_t hx = (L.geo.nx + 1) / 2;
        const int nb = nblk(hx * L.geo.ny * L.geo.nz);
        for (int s = 0; s < pre; ++s) {
            hipLaunchKernelGGL(k_mg_gs<T>, dim3(nb), dim3(CB), 0, c->stream, L.geo, cf, L.b, L.x, 0, s == 0 ? 1 : 0,
                               (const double *)nullptr, C.geo);
            hipLaunchKernelGGL(k_mg_gs<T>, dim3(nb), dim3(CB), 0, c->stream, L.geo, cf, L.b, L.x, 1, 0,
                               (const double *)nullptr, C.geo);
        }
        hipLaunchKernelGGL(k_mg_restrict<T>, dim3(nblk(C.n)), dim3(CB), 0, c->stream, L.geo, cf, L.b, L.x, C.geo,
                           C.b);
        RSV_LAUNCH(c);
        rsv_status st = cycle_t<T>(l + 1);
        if (st != RSV_OK) return st;
        for (int s = 0; s < post; ++s) {
            hipLaunchKernelGGL(k_mg_gs<T>, dim3(nb), dim3(CB), 0, c->stream, L.geo, cf, L.b, L.x, 1, 0,
                               s == 0 ? (const double *)C.x : (const double *)nullptr, C.geo);
            hipLaunchKernelGGL(k_mg_gs<T>, dim3(nb), dim3(CB), 0, c->stream, L.geo, cf, L.b, L.x, 0, 0,
                               (const double *)nullptr, C.geo);
        }
        RSV_LAUNCH(c);
        return RSV_OK;
    }

    // e = lev[0].x = M_g^-1 lev[0].b
    rsv_status pressure()
    {
        ProfScope ps(c, RSV_K_CPR);
        return cycle(0);
    }

    rsv_status resid(int mode, const double *x, const double *e, const double *f)
    {
        const Geo &g = A->g->geo;
        ProfScope ps(c, RSV_K_CPR);
        const dim3 grid(nblk(g.nslot)), blk(CB);
        if (fp32 && mode == 0)
            hipLaunchKernelGGL((k_cpr_resid<0, float>), grid, blk, 0, c->stream, g, (const float *)A32, x, e, f,
                               (double *)nullptr, (const double *)w, lev[0].b);
        else if (fp32)
            hipLaunchKernelGGL((k_cpr_resid<1, float>), grid, blk, 0, c->stream, g, (const float *)A32, x, e, f, r,
                               (const double *)w, (double *)nullptr);
        else if (mode == 0)
            hipLaunchKernelGGL((k_cpr_resid<0, double>), grid, blk, 0, c->stream, g, (const double *)A->d_A, x, e, f,
                               (double *)nullptr, (const double *)w, lev[0].b);
        else
            hipLaunchKernelGGL((k_cpr_resid<1, double>), grid, blk, 0, c->stream, g, (const double *)A->d_A, x, e, f,
                               r, (const double *)w, (double *)nullptr);
        RSV_LAUNCH(c);
        return RSV_OK;
    }

    // z_p += e: the pressure correction folded into z before the residual at
    // z + Pi_p e, which then reads no e (the same sums: x_p + e is formed in
    // FP64 either way)
    rsv_status prolong(double *z)
    {
        const Geo &g = A->g->geo;
        ProfScope ps(c, RSV_K_CPR);
        hipLaunchKernelGGL(k_cpr_prolong, dim3(nblk(g.nslot)), dim3(CB), 0, c->stream, g, z, (const double *)lev[0].x);
        RSV_LAUNCH(c);
        return RSV_OK;
    }

    rsv_status combine(double *z, const double *e, int has_z)
    {
        const Geo &g = A->g->geo;
        ProfScope ps(c, RSV_K_CPR);
        hipLaunchKernelGGL(k_cpr_combine, dim3(nblk(g.nslot)), dim3(CB), 0, c->stream, g, z, e, (const double *)t,
                           has_z);
        RSV_LAUNCH(c);
        return RSV_OK;
    }

    rsv_status apply(const double *f, double *z) override
    {
        const Geo &g = A->g->geo;
        const double *e = lev[0].x;
        rsv_status s = RSV_OK;
        switch (variant) {
        case RSV_CPR_FP:
            if ((s = R->apply(f, z)) != RSV_OK) return s;
            if ((s = resid(0, z, nullptr, f)) != RSV_OK) return s;
            if ((s = pressure()) != RSV_OK) return s;
            return prolong(z);
        case RSV_CPR_PF:
            {
                ProfScope ps(c, RSV_K_CPR);
                hipLaunchKernelGGL(k_cpr_restrict, dim3(nblk(g.nslot)), dim3(CB), 0, c->stream, g,
                                   (const double *)w, f, lev[0].b);
                RSV_LAUNCH(c);
            }
            if ((s = pressure()) != RSV_OK) return s;
            if ((s = resid(1, nullptr, e, f)) != RSV_OK) return s;
            if ((s = R->apply(r, t)) != RSV_OK) return s;
            return combine(z, e, 0);
        case RSV_CPR_FPF:
            if ((s = R->apply(f, z)) != RSV_OK) return s;
            if ((s = resid(0, z, nullptr, f)) != RSV_OK) return s;
            if ((s = pressure()) != RSV_OK) return s;
            if ((s = prolong(z)) != RSV_OK) return s;
            if ((s = resid(1, z, nullptr, f)) != RSV_OK) return s;
            if ((s = R->apply(r, t)) != RSV_OK) return s;
            return combine(z, nullptr, 1);
        case RSV_CPR_FFPF:
            if ((s = R->apply(f, z)) != RSV_OK) return s;
            if ((s = resid(1, z, nullptr, f)) != RSV_OK) return s;
            if ((s = R->apply(r, t)) != RSV_OK) return s;
            if ((s = combine(z, nullptr, 1)) != RSV_OK) return s;
            if ((s = resid(0, z, nullptr, f)) != RSV_OK) return s;
            if ((s = pressure()) != RSV_OK) return s;
            if ((s = prolong(z)) != RSV_OK) return s;
            if ((s = resid(1, z, nullptr, f)) != RSV_OK) return s;
            if ((s = R->apply(r, t)) != RSV_OK) return s;
            return combine(z, nullptr, 1);
        default: return set_err(c, RSV_ERR_ARG, "bad CPR variant");
        }
    }
};

template <>
const double *CprImpl::coef_of<double>(const MgLevel &L) { return L.coef; }
template <>
const float *CprImpl::coef_of<float>(const MgLevel &L) { return L.coef32; }

}  // namespace

rsv_status cpr_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl *stage, PcImpl **out, int64_t *bad_cell)
{
    rsv_ctx *c = A->g->ctx;
    if (p->cpr_variant < RSV_CPR_FP || p->cpr_variant > RSV_CPR_FFPF) {
        delete stage;
        return set_err(c, RSV_ERR_ARG, "bad CPR variant");
    }
    CprImpl *P = new (std::nothrow) CprImpl();
    if (!P) {
        delete stage;
        return set_err(c, RSV_ERR_OOM, "CPR preconditioner");
    }
    P->A = A;
    P->c = c;
    P->R = stage;
    P->variant = p->cpr_variant;
    P->pre = p->mg_pre;
    P->post = p->mg_post;
    P->fp32 = (p->precision == RSV_FP32);
    const Geo &g = A->g->geo;
    rsv_status s = RSV_OK;
    // levels: halve every axis longer than one cell until at most mg_coarse cells
    {
        MgLevel L0;
        L0.geo = LevelGeo{g.nx, g.ny, g.nz};
        L0.n = (int64_t)g.nx * g.ny * g.nz;
        P->lev.push_back(L0);
        while (P->lev.back().n > p->mg_coarse && P->lev.back().n > 1 && (int)P->lev.size() < MG_MAX_LEVELS) {
            const LevelGeo &f = P->lev.back().geo;
            MgLevel L;
            L.geo = LevelGeo{cdim(f.nx), cdim(f.ny), cdim(f.nz)};
            L.n = (int64_t)L.geo.nx * L.geo.ny * L.geo.nz;
            P->lev.push_back(L);
        }
        if (P->lev.back().n > p->mg_coarse) s = set_err(c, RSV_ERR_ARG, "multigrid hierarchy too deep");
    }
    const int64_t nv = A->g->nv;
    if (s == RSV_OK) s = P->alloc(&P->w, nv);
    if (s == RSV_OK) s = P->alloc(&P->r, nv);
    if (s == RSV_OK) s = P->alloc(&P->t, nv);
    // the work vectors' phantom slots stay zero whatever the stage R writes
    if (s == RSV_OK && (hipMemsetAsync(P->r, 0, (size_t)nv * 8, c->stream) != hipSuccess ||
                        hipMemsetAsync(P->t, 0, (size_t)nv * 8, c->stream) != hipSuccess))
        s = set_err(c, RSV_ERR_HIP, "hipMemsetAsync");
    for (auto &L : P->lev) {
        if (s == RSV_OK) s = P->alloc(&L.coef, 7 * L.n);
        if (s == RSV_OK) s = P->alloc(&L.b, L.n);
        if (s == RSV_OK) s = P->alloc(&L.x, L.n);
    }
    const int64_t nco = P->lev.back().n;
    double *aug = nullptr;
    if (s == RSV_OK) s = P->alloc(&P->inv, nco * nco);
    if (s == RSV_OK) s = dev_alloc(c, (void **)&aug, (size_t)(2 * nco * nco) * 8);
    if (s == RSV_OK) s = flags_reset(c);
    if (s == RSV_OK) {
        ProfScope ps(c, RSV_K_FACTOR);
        hipLaunchKernelGGL(k_cpr_extract, dim3(nblk(g.nslot)), dim3(CB), 0, c->stream, g, (const double *)A->d_A,
                           p->cpr_decouple, P->w, P->lev[0].coef, c->d_flags);
        for (size_t l = 0; l + 1 < P->lev.size(); ++l)
            hipLaunchKernelGGL(k_mg_galerkin, dim3(nblk(P->lev[l + 1].n)), dim3(CB), 0, c->stream, P->lev[l].geo,
                               (const double *)P->lev[l].coef, P->lev[l + 1].geo, P->lev[l + 1].coef);
        for (size_t l = 0; l < P->lev.size(); ++l)
            hipLaunchKernelGGL(k_mg_check, dim3(nblk(P->lev[l].n)), dim3(CB), 0, c->stream, P->lev[l].n,
                               (const double *)P->lev[l].coef, (int)l, c->d_flags);
        const MgLevel &Lc = P->lev.back();
        hipLaunchKernelGGL(k_mg_dense, dim3(nblk(Lc.n)), dim3(CB), 0, c->stream, Lc.geo, (const double *)Lc.coef,
                           aug);
        hipLaunchKernelGGL(k_mg_gauss_jordan, dim3(1), dim3(GJ_T), 0, c->stream, (int)Lc.n, aug, P->inv,
                           c->d_flags);
        if (P->fp32) {
            // FP32 form: the residual products and the cycle read FP32 copies
            const int64_t na = 63 * g.nslot;
            P->nbytes += na * 4;
            if ((s = dev_alloc(c, (void **)&P->A32, (size_t)na * 4)) == RSV_OK)
                hipLaunchKernelGGL(k_to_f32, dim3(nblk(na)), dim3(CB), 0, c->stream, na, (const double *)A->d_A,
                                   P->A32);
            for (auto &L : P->lev) {
                if (s != RSV_OK) break;
                P->nbytes += 7 * L.n * 4;
                if ((s = dev_alloc(c, (void **)&L.coef32, (size_t)(7 * L.n) * 4)) == RSV_OK)
                    hipLaunchKernelGGL(k_to_f32, dim3(nblk(7 * L.n)), dim3(CB), 0, c->stream, 7 * L.n,
                                       (const double *)L.coef, L.coef32);
            }
        }
        hipError_t e = hipGetLastError();
        if (s == RSV_OK && e != hipSuccess)
            s = set_err(c, RSV_ERR_HIP, std::string("CPR setup launch: ") + hipGetErrorString(e));
    }
    if (s == RSV_OK) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) s = set_err(c, RSV_ERR_HIP, std::string("sync: ") + hipGetErrorString(e));
    }
    dev_free(aug);
    if (s == RSV_OK) s = flags_check(c, bad_cell);
    if (s != RSV_OK) {
        delete P;
        return s;
    }
    *out = P;
    return RSV_OK;
}

// diagnostics ------------------------------------------------------------

static CprImpl *cpr_of(const rsv_precond *M)
{
    if (!M || M->p.type != RSV_PC_CPR || !M->impl) return nullptr;
    return static_cast<CprImpl *>(M->impl);
}

extern "C" {

rsv_status rsv_cpr_levels(const rsv_precond *M, int32_t *nlevels, int32_t *dims, int32_t cap)
{
    CprImpl *P = cpr_of(M);
    if (!P || !nlevels || cap < 0 || (cap > 0 && !dims))
        return set_err(M ? M->A->g->ctx : nullptr, RSV_ERR_ARG, "not a CPR preconditioner or bad argument");
    *nlevels = (int32_t)P->lev.size();
    for (int l = 0; l < (int)P->lev.size() && l < cap; ++l) {
        dims[3 * l] = P->lev[l].geo.nx;
        dims[3 * l + 1] = P->lev[l].geo.ny;
        dims[3 * l + 2] = P->lev[l].geo.nz;
    }
    return RSV_OK;
}

rsv_status rsv_cpr_pressure_matrix(const rsv_precond *M, int32_t level, double *coef)
{
    CprImpl *P = cpr_of(M);
    if (!P || !coef || level < 0 || level >= (int)P->lev.size())
        return set_err(M ? M->A->g->ctx : nullptr, RSV_ERR_ARG, "not a CPR preconditioner or bad level");
    rsv_ctx *c = P->c;
    const MgLevel &L = P->lev[level];
    std::vector<double> tmp((size_t)(7 * L.n));
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    RSV_HIP(c, hipMemcpy(tmp.data(), L.coef, (size_t)(7 * L.n) * 8, hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < L.n; ++r)
        for (int d = 0; d < 7; ++d) coef[7 * r + d] = tmp[(size_t)(d * L.n + r)];
    return RSV_OK;
}

rsv_status rsv_cpr_weights(const rsv_precond *M, double *w)
{
    CprImpl *P = cpr_of(M);
    if (!P || !w) return set_err(M ? M->A->g->ctx : nullptr, RSV_ERR_ARG, "not a CPR preconditioner or bad argument");
    rsv_ctx *c = P->c;
    const rsv_grid *g = P->A->g;
    double *nat = nullptr;
    rsv_status s = dev_alloc(c, (void **)&nat, (size_t)(3 * g->ncell) * 8);
    if (s == RSV_OK) s = launch_tl_to_nat(c, g->geo, P->w, nat, 1.0, 0.0);
    if (s == RSV_OK) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) e = hipMemcpy(w, nat, (size_t)(3 * g->ncell) * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) s = set_err(c, RSV_ERR_HIP, std::string("weights: ") + hipGetErrorString(e));
    }
    dev_free(nat);
    return s;
}

rsv_status rsv_cpr_pressure_apply(rsv_precond *M, const double *b, double *x)
{
    CprImpl *P = cpr_of(M);
    if (!P || !b || !x || b == x)
        return set_err(M ? M->A->g->ctx : nullptr, RSV_ERR_ARG, "not a CPR preconditioner or bad argument");
    rsv_ctx *c = P->c;
    const int64_t n = P->lev[0].n;
    rsv_status s = launch_copy(c, n, b, P->lev[0].b);
    if (s == RSV_OK) s = P->pressure();
    if (s == RSV_OK) s = launch_copy(c, n, P->lev[0].x, x);
    if (s == RSV_OK) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) s = set_err(c, RSV_ERR_HIP, std::string("sync: ") + hipGetErrorString(e));
    }
    return s;
}

}  // extern "C"
