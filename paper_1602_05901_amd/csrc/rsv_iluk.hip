// ILU(k) local solvers for restricted additive Schwarz (the ILUK local
// solver of the RAS data structure and its level parameter, Restricted
// Additive Schwarz Method subsection), for 3x3-block matrices.
//
// Subdomains, overlap and owner-only write-back are those of the ILU(0) RAS:
// px x py x pz boxes (the first n mod p one cell longer), Omega_s = the cells
// within graph distance `overlap` of the box, local order = ascending global
// (bottom-up natural) index.  ILU(k) keeps the fill positions whose level of
// fill is at most k: the stencil positions have level 0, and eliminating row
// m from row i gives (i, j) the level lev(i,m) + lev(m,j) + 1.  With fill
// the hyperplane schedule of ILU(0) no longer holds (level-1 fill couples
// cell c to c + e_x - e_y, a cell of the same plane i + j + k), so rows are
// scheduled by dependency levels computed from the symbolic pattern: a row's
// forward level is one more than that of every column of its L part, its
// backward level one more than that of every column of its U part.
//
// Host: the symbolic factorisation and the schedules, per subdomain (threads
// over subdomains).  Device: one workgroup per subdomain walks its levels
// with a barrier between them -- the IKJ numeric factorisation (a row's L
// blocks times the inverted pivots of the rows they reference, each update
// merged into the row's sorted pattern, then the row's own pivot inverted by
// cofactors), and for an apply the forward sweep y_i = r_i - sum L_ij y_j and
// the backward sweep z_i = U_ii^-1 (y_i - sum U_ij z_j), the owner writing
// z_i into the tile-lane result.
//
// ILUT(p, tol) local solvers (the RAS parameters' ILUT solver) share the
// subdomains and the apply; their factorisation and schedules run on the
// device (see the ILUT section below).
#include "rsv_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <new>
#include <thread>
#include <vector>

namespace {

constexpr int KT = 256;   // threads of a subdomain's workgroup (factorisation)
constexpr int KA = 1024;  // threads of a subdomain's workgroup (apply: a level's rows spread over more lanes)

struct IlukDev {
    int64_t nrow;
    const int32_t *gslot, *own;          // per row: tile-lane slot of its cell; 1 if the subdomain owns it
    const int64_t *lptr, *uptr;          // per row: first entry in the L / U position arrays
    const int64_t *lend, *uend;          // per row: one past its last entry (ILU(k): lptr + 1, uptr + 1)
    const int32_t *lcol, *ucol;          // column = row index (global across subdomains)
    const int64_t *lsrc, *usrc;          // A-entry base index of a stencil position, -1 for fill
    double *lval, *uval, *dval, *dinv;   // 9 per position / row, row-major blocks
    double *y;                           // 3 per row
    const int32_t *fo, *bo;              // rows in forward / backward level order
    const int64_t *fl, *bl;              // level boundaries into fo / bo
    const int32_t *fl_off, *bl_off, *fl_cnt, *bl_cnt;   // per subdomain: first boundary, level count
    const int64_t *dbase;                // per row: A-entry base index of the diagonal block
};

__device__ inline void mm3_sub(const double *a, const double *b, double *c)   // c -= a b
{
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) c[3 * p + q] -= a[3 * p] * b[q] + a[3 * p + 1] * b[3 + q] + a[3 * p + 2] * b[6 + q];
}

// initial values: the blocks of A at stencil positions (tile-lane entries
// 64 apart), zero at fill positions
__global__ __launch_bounds__(256) void k_iluk_load(const double *__restrict__ A, IlukDev d, int64_t nl, int64_t nu)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t tot = nl + nu + d.nrow;
    if (t >= tot) return;
    int64_t src;
    double *dst;
    if (t < nl) { src = d.lsrc[t]; dst = d.lval + 9 * t; }
    else if (t < nl + nu) { src = d.usrc[t - nl]; dst = d.uval + 9 * (t - nl); }
    else { src = d.dbase[t - nl - nu]; dst = d.dval + 9 * (t - nl - nu); }
#pragma unroll
    for (int e = 0; e < 9; ++e) dst[e] = (src >= 0) ? A[src + 64 * e] : 0.0;
}

__global__ __launch_bounds__(KT) void k_iluk_factor(IlukDev d, int32_t *flags)
{
    const int s = blockIdx.x;
    const int nlev = d.fl_cnt[s];
    const int64_t *fl = d.fl + d.fl_off[s];
    for (int lv = 0; lv < nlev; ++lv) {
        for (int64_t t = fl[lv] + threadIdx.x; t < fl[lv + 1]; t += KT) {
            const int32_t i = d.fo[t];
            const int64_t l0 = d.lptr[i], l1 = d.lptr[i + 1], u0 = d.uptr[i], u1 = d.uptr[i + 1];
            for (int64_t p = l0; p < l1; ++p) {
                const int32_t k = d.lcol[p];
                double lik[9], a[9];
#pragma unroll
                for (int e = 0; e < 9; ++e) a[e] = d.lval[9 * p + e];
                const double *dk = d.dinv + 9 * k;
#pragma unroll
                for (int pp = 0; pp < 3; ++pp)
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        lik[3 * pp + q] = a[3 * pp] * dk[q] + a[3 * pp + 1] * dk[3 + q] + a[3 * pp + 2] * dk[6 + q];
#pragma unroll
                for (int e = 0; e < 9; ++e) d.lval[9 * p + e] = lik[e];
                // row i -= L_ik (row k's U part), merged into the sorted pattern of row i
                int64_t pl = p + 1, pu = u0;
                for (int64_t q = d.uptr[k]; q < d.uptr[k + 1]; ++q) {
                    const int32_t j = d.ucol[q];
                    double *tgt = nullptr;
                    if (j < i) {
                        while (pl < l1 && d.lcol[pl] < j) ++pl;
                        if (pl < l1 && d.lcol[pl] == j) tgt = d.lval + 9 * pl;
                    } else if (j == i) {
                        tgt = d.dval + 9 * (int64_t)i;
                    } else {
                        while (pu < u1 && d.ucol[pu] < j) ++pu;
                        if (pu < u1 && d.ucol[pu] == j) tgt = d.uval + 9 * pu;
                    }
                    if (tgt) mm3_sub(lik, d.uval + 9 * q, tgt);
                }
            }
            double D[9], Di[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) D[e] = d.dval[9 * (int64_t)i + e];
            if (!inv3(D, Di)) {
                atomicOr(&flags[0], (int32_t)FLAG_PIVOT);
                atomicMin(&flags[1], (int32_t)d.own[i] >> 1);   // the row's cell, stored with the owner bit
#pragma unroll
                for (int e = 0; e < 9; ++e) Di[e] = 0.0;
            }
#pragma unroll
            for (int e = 0; e < 9; ++e) d.dinv[9 * (int64_t)i + e] = Di[e];
        }
        __syncthreads();
    }
}

// One row of the forward sweep, y_i = r_i - sum L_ij y_j: the blocks and y
// values of up to four entries are loaded before their products are
// subtracted (in entry order).
__device__ inline void iluk_fwd_row(const IlukDev &d, const double *__restrict__ r, int32_t i)
{
    const int64_t sl = d.gslot[i];
    double v0 = r[vidx(sl, 0)], v1 = r[vidx(sl, 1)], v2 = r[vidx(sl, 2)];
    const int64_t pe = d.lend[i];
    for (int64_t p0 = d.lptr[i]; p0 < pe; p0 += 4) {
        double L[4][9], y[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (p0 + q >= pe) continue;
            const double *Lp = d.lval + 9 * (p0 + q), *yk = d.y + 3 * (int64_t)d.lcol[p0 + q];
#pragma unroll
            for (int e = 0; e < 9; ++e) L[q][e] = Lp[e];
#pragma unroll
            for (int e = 0; e < 3; ++e) y[q][e] = yk[e];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (p0 + q >= pe) continue;
            v0 -= L[q][0] * y[q][0] + L[q][1] * y[q][1] + L[q][2] * y[q][2];
            v1 -= L[q][3] * y[q][0] + L[q][4] * y[q][1] + L[q][5] * y[q][2];
            v2 -= L[q][6] * y[q][0] + L[q][7] * y[q][1] + L[q][8] * y[q][2];
        }
    }
    d.y[3 * (int64_t)i] = v0;
    d.y[3 * (int64_t)i + 1] = v1;
    d.y[3 * (int64_t)i + 2] = v2;
}

// One row of the backward sweep, z_i = U_ii^-1 (y_i - sum U_ij z_j) (z in
// place of y), the owner also writing z_i into the tile-lane result.
__device__ inline void iluk_bwd_row(const IlukDev &d, double *__restrict__ z, int32_t i)
{
    double v0 = d.y[3 * (int64_t)i], v1 = d.y[3 * (int64_t)i + 1], v2 = d.y[3 * (int64_t)i + 2];
    const int64_t qe = d.uend[i];
    for (int64_t q0 = d.uptr[i]; q0 < qe; q0 += 4) {
        double U[4][9], w[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q0 + q >= qe) continue;
            const double *Uq = d.uval + 9 * (q0 + q), *zj = d.y + 3 * (int64_t)d.ucol[q0 + q];
#pragma unroll
            for (int e = 0; e < 9; ++e) U[q][e] = Uq[e];
#pragma unroll
            for (int e = 0; e < 3; ++e) w[q][e] = zj[e];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q0 + q >= qe) continue;
            v0 -= U[q][0] * w[q][0] + U[q][1] * w[q][1] + U[q][2] * w[q][2];
            v1 -= U[q][3] * w[q][0] + U[q][4] * w[q][1] + U[q][5] * w[q][2];
            v2 -= U[q][6] * w[q][0] + U[q][7] * w[q][1] + U[q][8] * w[q][2];
        }
    }
    const double *Di = d.dinv + 9 * (int64_t)i;
    const double w0 = Di[0] * v0 + Di[1] * v1 + Di[2] * v2;
    const double w1 = Di[3] * v0 + Di[4] * v1 + Di[5] * v2;
    const double w2 = Di[6] * v0 + Di[7] * v1 + Di[8] * v2;
    d.y[3 * (int64_t)i] = w0;
    d.y[3 * (int64_t)i + 1] = w1;
    d.y[3 * (int64_t)i + 2] = w2;
    if (d.own[i] & 1) {
        const int64_t sl = d.gslot[i];
        z[vidx(sl, 0)] = w0;
        z[vidx(sl, 1)] = w1;
        z[vidx(sl, 2)] = w2;
    }
}

// Small subdomains: one workgroup per subdomain walks its levels.
__global__ __launch_bounds__(KA) void k_iluk_apply(IlukDev d, const double *__restrict__ r, double *__restrict__ z)
{
    const int s = blockIdx.x;
    {
        const int nlev = d.fl_cnt[s];
        const int64_t *fl = d.fl + d.fl_off[s];
        for (int lv = 0; lv < nlev; ++lv) {
            for (int64_t t = fl[lv] + threadIdx.x; t < fl[lv + 1]; t += KA) iluk_fwd_row(d, r, d.fo[t]);
            __syncthreads();
        }
    }
    {
        const int nlev = d.bl_cnt[s];
        const int64_t *bl = d.bl + d.bl_off[s];
        for (int lv = 0; lv < nlev; ++lv) {
            for (int64_t t = bl[lv] + threadIdx.x; t < bl[lv + 1]; t += KA) iluk_bwd_row(d, z, d.bo[t]);
            __syncthreads();
        }
    }
}

// Large subdomains: one launch per level of every subdomain at once
// (grid.y = subdomain, grid.x workgroups striding over the level's rows), so
// the whole chip works on a level and the kernel boundary orders the levels.
constexpr int LV_WG = 4;   // workgroups per subdomain and level
__global__ __launch_bounds__(256) void k_iluk_fwd_level(IlukDev d, const double *__restrict__ r, int lv)
{
    const int s = blockIdx.y;
    if (lv >= d.fl_cnt[s]) return;
    const int64_t *fl = d.fl + d.fl_off[s];
    for (int64_t t = fl[lv] + blockIdx.x * 256 + threadIdx.x; t < fl[lv + 1]; t += (int64_t)gridDim.x * 256)
        iluk_fwd_row(d, r, d.fo[t]);
}
__global__ __launch_bounds__(256) void k_iluk_bwd_level(IlukDev d, double *__restrict__ z, int lv)
{
    const int s = blockIdx.y;
    if (lv >= d.bl_cnt[s]) return;
    const int64_t *bl = d.bl + d.bl_off[s];
    for (int64_t t = bl[lv] + blockIdx.x * 256 + threadIdx.x; t < bl[lv + 1]; t += (int64_t)gridDim.x * 256)
        iluk_bwd_row(d, z, d.bo[t]);
}

// The apply of either form: per-level launches when a level has at least 256
// rows per subdomain on average, else one workgroup per subdomain.
inline rsv_status iluk_apply(rsv_ctx *c, const IlukDev &d, int nsub, int nfl_max, int nbl_max, bool per_level,
                             const double *r, double *z)
{
    if (!per_level) {
        hipLaunchKernelGGL(k_iluk_apply, dim3(nsub), dim3(KA), 0, c->stream, d, r, z);
        RSV_LAUNCH(c);
        return RSV_OK;
    }
    const dim3 grid(LV_WG, nsub);
    for (int lv = 0; lv < nfl_max; ++lv) hipLaunchKernelGGL(k_iluk_fwd_level, grid, dim3(256), 0, c->stream, d, r, lv);
    for (int lv = 0; lv < nbl_max; ++lv) hipLaunchKernelGGL(k_iluk_bwd_level, grid, dim3(256), 0, c->stream, d, z, lv);
    RSV_LAUNCH(c);
    return RSV_OK;
}

// ---------------------------------------------------------------- ILUT(p, tol)
//
// Threshold ILU with 3x3 blocks (the RAS parameters' ILUT solver, ilut_p and
// ilut_tol), Saad's row-wise ILUT with blocks measured by their squared
// Frobenius norm: row i starts as block row i of A with the threshold
// thr = tol^2 * sum |A_ij|^2; its positions left of i are eliminated in
// ascending order (w_k <- w_k U_kk^-1, dropped when |w_k|^2 < thr, else
// w <- w - w_k U_k,:), fill entering as it is created; the positions right
// of i below thr are dropped; the p largest left and right of i are kept
// (ties: smaller column first; p < 0: as many as A's row holds on that
// side); U_ii^-1 by LU with partial pivoting.
//
// The pattern depends on the values, so everything runs on the device: one
// wavefront per subdomain factors its rows in order.  The work row lives in
// LDS: a map from column (mod the window length 2 bw + 1, bw = the local
// band width) to a slot of a small block buffer, a sorted list of the
// positions still to eliminate, and per slot the block and whether it was
// dropped.  The floating-point steps run in the oracle's order without
// contraction (products sum their three terms left to right, norms their
// nine squares in order, the pivot inverse is the same textbook LU), so the
// drop and keep decisions are the oracle's.  Afterwards the same wavefront
// computes the dependency levels (forward from the kept L columns, backward
// from the kept U columns) and buckets its rows by level for the apply of
// the ILU(k) path (k_iluk_apply).

constexpr int TW = 64;            // one wavefront per subdomain
constexpr int T_NBUF = 512;       // blocks of the work row
constexpr int T_LCAP = 512;       // positions left of i awaiting elimination
constexpr int T_CAP_MAX = 32;     // largest p
constexpr int FLAG_ILUT_CAP = 16; // a row needed more than T_NBUF / T_LCAP entries

struct IlutDev {
    int64_t nrow;
    const int32_t *acol;          // [nrow][7] global row of the stencil column, -1 outside Omega_s
    const int64_t *asrc;          // [nrow][7] A entry base index of that block
    const int64_t *sub_base;      // nsub + 1
    const int32_t *sub_w;         // window length per subdomain
    const int32_t *own;           // row of the cell << 1 | owner bit
    int32_t p, capl, capu;
    double tol2;
    const int64_t *lptr, *uptr;   // row capacity starts
    int64_t *lend, *uend;
    int32_t *lcol, *ucol;
    double *lval, *uval, *dval, *dinv;
    int32_t *flev, *blev;
    int32_t *fo, *bo;
    int64_t *fl, *bl;             // per subdomain boundaries at fl_off[s] = base[s] + s
    int32_t *fl_cnt, *bl_cnt;
    int64_t *cnt;                 // scratch, same layout as fl
    int64_t *nkept;               // per subdomain: L and U blocks kept
};

__device__ inline double fro2_blk(const double *a)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int e = 0; e < 9; ++e) s = s + a[e] * a[e];
    return s;
}

__device__ inline void blk_mul_t(const double *a, const double *b, double *c)   // c = a b
{
#pragma clang fp contract(off)
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            double t = a[3 * p] * b[q];
            t = t + a[3 * p + 1] * b[3 + q];
            t = t + a[3 * p + 2] * b[6 + q];
            c[3 * p + q] = t;
        }
}

__device__ inline double norm1_blk(const double *a)
{
    double best = 0.0;
    for (int q = 0; q < 3; ++q) {
        double s = fabs(a[q]) + fabs(a[3 + q]);
        s = s + fabs(a[6 + q]);
        if (s > best) best = s;
    }
    return best;
}

// inverse by LU with partial pivoting, solving for the three unit vectors;
// a pivot |u_pp| <= 1e-300 or a 1-norm condition above 1e14 is singular
__device__ inline bool inv3_lu(const double *a, double *o)
{
#pragma clang fp contract(off)
    double lu[9];
    int perm[3] = {0, 1, 2};
    for (int e = 0; e < 9; ++e) lu[e] = a[e];
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(lu[3 * r + c]) > fabs(lu[3 * piv + c])) piv = r;
        if (!(fabs(lu[3 * piv + c]) > 1e-300)) return false;
        if (piv != c) {
            for (int q = 0; q < 3; ++q) {
                const double t = lu[3 * c + q];
                lu[3 * c + q] = lu[3 * piv + q];
                lu[3 * piv + q] = t;
            }
            const int t = perm[c];
            perm[c] = perm[piv];
            perm[piv] = t;
        }
        for (int r = c + 1; r < 3; ++r) {
            const double f = lu[3 * r + c] / lu[3 * c + c];
            lu[3 * r + c] = f;
            for (int q = c + 1; q < 3; ++q) lu[3 * r + q] = lu[3 * r + q] - f * lu[3 * c + q];
        }
    }
    for (int col = 0; col < 3; ++col) {
        double y[3];
        for (int r = 0; r < 3; ++r) {
            double v = (perm[r] == col) ? 1.0 : 0.0;
            for (int t = 0; t < r; ++t) v = v - lu[3 * r + t] * y[t];
            y[r] = v;
        }
        for (int r = 2; r >= 0; --r) {
            double v = y[r];
            for (int t = r + 1; t < 3; ++t) v = v - lu[3 * r + t] * o[3 * t + col];
            o[3 * r + col] = v / lu[3 * r + r];
        }
    }
    return norm1_blk(a) * norm1_blk(o) <= 1e14;
}

// wavefront-wide inclusive prefix sum of v
__device__ inline int64_t wave_scan(int64_t v)
{
    const int lane = threadIdx.x & 63;
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

// rows of [g0, g1) bucketed by level lev[] (nlev levels): bounds and order
__device__ void bucket_rows(int64_t g0, int64_t g1, const int32_t *lev, int nlev, int64_t *cnt, int64_t *bounds,
                            int32_t *ord)
{
    const int lane = threadIdx.x;
    for (int l = lane; l <= nlev; l += TW) cnt[l] = 0;
    __syncthreads();
    for (int64_t g = g0 + lane; g < g1; g += TW) atomicAdd((unsigned long long *)&cnt[lev[g]], 1ull);
    __syncthreads();
    // exclusive scan of cnt[0..nlev) into bounds, offset g0
    int64_t carry = 0;
    for (int l0 = 0; l0 < nlev; l0 += TW) {
        const int l = l0 + lane;
        const int64_t v = (l < nlev) ? cnt[l] : 0;
        const int64_t inc = wave_scan(v);
        if (l < nlev) bounds[l] = g0 + carry + inc - v;
        carry += __shfl(inc, 63, 64);
    }
    if (lane == 0) bounds[nlev] = g0 + carry;
    __syncthreads();
    for (int l = lane; l < nlev; l += TW) cnt[l] = bounds[l];
    __syncthreads();
    for (int64_t g = g0 + lane; g < g1; g += TW) {
        const int64_t at = (int64_t)atomicAdd((unsigned long long *)&cnt[lev[g]], 1ull);
        ord[at] = (int32_t)g;
    }
    __syncthreads();
}

__global__ __launch_bounds__(TW) void k_ilut_factor(IlutDev t, const double *__restrict__ A, int32_t *flags)
{
#pragma clang fp contract(off)
    extern __shared__ __align__(16) unsigned char smem[];
    const int s = blockIdx.x, lane = threadIdx.x;
    const int64_t g0 = t.sub_base[s], g1 = t.sub_base[s + 1];
    const int32_t W = t.sub_w[s];
    double *wbuf = (double *)smem;                       // [T_NBUF][9]
    double *cf2 = wbuf + 9 * T_NBUF;                     // [T_NBUF] squared norms
    int32_t *touched = (int32_t *)(cf2 + T_NBUF);        // [T_NBUF] column of each slot
    int32_t *llist = touched + T_NBUF;                   // [T_LCAP]
    int32_t *tslot = llist + T_LCAP;                     // [T_CAP_MAX]
    int32_t *outpos = tslot + T_CAP_MAX;                 // [T_NBUF] output position of a kept slot, -1 none
    unsigned char *cls = (unsigned char *)(outpos + T_NBUF);   // [T_NBUF] 0 none, 1 L, 2 U, 3 diagonal
    unsigned char *dropped = cls + T_NBUF;               // [T_NBUF]
    int16_t *wmap = (int16_t *)(dropped + T_NBUF);       // [W]
    __shared__ double wk[9], thr_s;
    __shared__ int nbuf, nll, pos_s, keep_s, nu_s, err_s, nla_s, nua_s, maxf_s, nkl_s, nku_s, diag_s;
    __shared__ unsigned long long kept_s;
    __shared__ int64_t q0_s;

    for (int q = lane; q < W; q += TW) wmap[q] = -1;
    if (lane == 0) { err_s = 0; maxf_s = 0; kept_s = 0; }
    __syncthreads();
    for (int64_t g = g0; g < g1; ++g) {
        // the row of A: slots 0.. in column (= stencil slot) order
        if (lane == 0) {
            nbuf = 0;
            nll = 0;
            int nla = 0, nua = 0;
            for (int st = 0; st < 7; ++st) {
                const int32_t c = t.acol[7 * g + st];
                if (c < 0) continue;
                const int sl = nbuf++;
                touched[sl] = c;
                dropped[sl] = 0;
                wmap[c % W] = (int16_t)sl;
                if (c < g) { llist[nll++] = c; ++nla; }
                if (c > g) ++nua;
            }
            nla_s = nla;
            nua_s = nua;
        }
        __syncthreads();
        for (int it = lane; it < 63; it += TW) {
            const int st = it / 9, e = it - 9 * (it / 9);
            const int32_t c = t.acol[7 * g + st];
            if (c >= 0) wbuf[9 * wmap[c % W] + e] = A[t.asrc[7 * g + st] + 64 * e];
        }
        __syncthreads();
        if (lane == 0) {
            double nrm2 = 0.0;
            for (int sl = 0; sl < nbuf; ++sl) nrm2 = nrm2 + fro2_blk(wbuf + 9 * sl);
            thr_s = t.tol2 * nrm2;
            pos_s = 0;
        }
        __syncthreads();
        // elimination of the positions left of g in ascending order
        for (;;) {
            if (pos_s >= nll || err_s) break;
            if (lane == 0) {
                const int32_t k = llist[pos_s];
                const int sk = wmap[k % W];
                double v[9];
                blk_mul_t(wbuf + 9 * sk, t.dinv + 9 * (int64_t)k, v);
                if (fro2_blk(v) < thr_s) {
                    dropped[sk] = 1;
                    keep_s = 0;
                } else {
                    for (int e = 0; e < 9; ++e) { wbuf[9 * sk + e] = v[e]; wk[e] = v[e]; }
                    keep_s = 1;
                    const int64_t q0 = t.uptr[k], q1 = t.uend[k];
                    q0_s = q0;
                    nu_s = (int)(q1 - q0);
                    for (int64_t q = q0; q < q1; ++q) {
                        const int32_t j = t.ucol[q];
                        int sl = wmap[j % W];
                        if (sl < 0) {
                            if (nbuf == T_NBUF) { err_s = 1; break; }
                            sl = nbuf++;
                            touched[sl] = j;
                            dropped[sl] = 0;
                            for (int e = 0; e < 9; ++e) wbuf[9 * sl + e] = 0.0;
                            wmap[j % W] = (int16_t)sl;
                            if (j < g) {
                                if (nll == T_LCAP) { err_s = 1; break; }
                                int at = nll++;
                                while (at > pos_s + 1 && llist[at - 1] > j) { llist[at] = llist[at - 1]; --at; }
                                llist[at] = j;
                            }
                        }
                        tslot[q - q0] = sl;
                    }
                }
                pos_s = pos_s + 1;
            }
            __syncthreads();
            if (keep_s && !err_s) {
                for (int it = lane; it < 9 * nu_s; it += TW) {
                    const int qq = it / 9, e = it - 9 * (it / 9), pp = e / 3, q3 = e - 3 * (e / 3);
                    const double *U = t.uval + 9 * (q0_s + qq);
                    double sacc = wk[3 * pp] * U[q3];
                    sacc = sacc + wk[3 * pp + 1] * U[3 + q3];
                    sacc = sacc + wk[3 * pp + 2] * U[6 + q3];
                    double *tgt = wbuf + 9 * tslot[qq] + e;
                    *tgt = *tgt - sacc;
                }
            }
            __syncthreads();
        }
        if (err_s) break;
        // classify the slots, then keep the largest of each side
        for (int sl = lane; sl < nbuf; sl += TW) {
            const int32_t c = touched[sl];
            const double f2 = fro2_blk(wbuf + 9 * sl);
            cf2[sl] = f2;
            unsigned char k = 0;
            if (c == g) k = 3;
            else if (!dropped[sl] && c < g) k = 1;
            else if (!dropped[sl] && c > g && !(f2 < thr_s)) k = 2;
            cls[sl] = k;
            outpos[sl] = -1;
        }
        __syncthreads();
        {
            const int pl = t.p < 0 ? nla_s : t.p, pu = t.p < 0 ? nua_s : t.p;
            // rank by size within the side (outpos holds it until the cut)
            for (int a = lane; a < nbuf; a += TW) {
                const int ka = cls[a];
                if (ka == 1 || ka == 2) {
                    int rank = 0;
                    for (int b = 0; b < nbuf; ++b)
                        if (b != a && cls[b] == ka &&
                            (cf2[b] > cf2[a] || (cf2[b] == cf2[a] && touched[b] < touched[a])))
                            ++rank;
                    outpos[a] = rank;
                }
            }
            __syncthreads();
            for (int a = lane; a < nbuf; a += TW) {
                const int ka = cls[a];
                if ((ka == 1 && outpos[a] >= pl) || (ka == 2 && outpos[a] >= pu)) cls[a] = 0;
            }
            __syncthreads();
            for (int a = lane; a < nbuf; a += TW) {
                const int ka = cls[a];
                if (ka == 1 || ka == 2) {
                    int r = 0;
                    for (int b = 0; b < nbuf; ++b)
                        if (cls[b] == ka && touched[b] < touched[a]) ++r;
                    outpos[a] = r;
                }
                if (ka == 3) diag_s = a;
            }
            __syncthreads();
            if (lane == 0) {
                int nkl = 0, nku = 0;
                for (int a = 0; a < nbuf; ++a) {
                    if (cls[a] == 1) ++nkl;
                    if (cls[a] == 2) ++nku;
                }
                nkl_s = nkl;
                nku_s = nku;
            }
            __syncthreads();
            // write the kept blocks in ascending column order
            for (int it = lane; it < 9 * nbuf; it += TW) {
                const int a = it / 9, e = it - 9 * (it / 9);
                const int ka = cls[a];
                if (ka == 1) {
                    const int64_t q = t.lptr[g] + outpos[a];
                    t.lval[9 * q + e] = wbuf[9 * a + e];
                    if (e == 0) t.lcol[q] = touched[a];
                } else if (ka == 2) {
                    const int64_t q = t.uptr[g] + outpos[a];
                    t.uval[9 * q + e] = wbuf[9 * a + e];
                    if (e == 0) t.ucol[q] = touched[a];
                } else if (ka == 3) {
                    t.dval[9 * g + e] = wbuf[9 * a + e];
                }
            }
        }
        if (lane == 0) {
            t.lend[g] = t.lptr[g] + nkl_s;
            t.uend[g] = t.uptr[g] + nku_s;
            kept_s += (unsigned long long)(nkl_s + nku_s);
            double di[9];
            if (!inv3_lu(wbuf + 9 * diag_s, di)) {
                atomicOr(&flags[0], (int32_t)FLAG_PIVOT);
                atomicMin(&flags[1], (int32_t)(t.own[g] >> 1));
                for (int e = 0; e < 9; ++e) di[e] = 0.0;
            }
            for (int e = 0; e < 9; ++e) t.dinv[9 * g + e] = di[e];
            // forward level: one more than every kept L column's
            int lv = 0;
            for (int a = 0; a < nbuf; ++a)
                if (cls[a] == 1) lv = max(lv, t.flev[touched[a]] + 1);
            t.flev[g] = lv;
            maxf_s = max(maxf_s, lv);
        }
        __syncthreads();
        for (int sl = lane; sl < nbuf; sl += TW) wmap[touched[sl] % W] = -1;
        __syncthreads();
    }
    if (err_s) {
        if (lane == 0) atomicOr(&flags[0], FLAG_ILUT_CAP);
        return;
    }
    // backward levels, descending rows
    __shared__ int maxb_s;
    if (lane == 0) {
        int mb = 0;
        for (int64_t g = g1 - 1; g >= g0; --g) {
            int lv = 0;
            for (int64_t q = t.uptr[g]; q < t.uend[g]; ++q) lv = max(lv, t.blev[t.ucol[q]] + 1);
            t.blev[g] = lv;
            mb = max(mb, lv);
        }
        maxb_s = mb;
        t.nkept[s] = (int64_t)kept_s;
        t.fl_cnt[s] = maxf_s + 1;
        t.bl_cnt[s] = mb + 1;
    }
    __syncthreads();
    const int64_t off = g0 + s;
    bucket_rows(g0, g1, t.flev, maxf_s + 1, t.cnt + off, t.fl + off, t.fo);
    bucket_rows(g0, g1, t.blev, maxb_s + 1, t.cnt + off, t.bl + off, t.bo);
}

int64_t kbox_start(int64_t b, int64_t len, int64_t p)
{
    const int64_t base = len / p, rem = len % p;
    return b * base + std::min(b, rem);
}

// Omega_s of subdomain s: the cells within graph distance ov of its box, in
// ascending global index, whether s owns each, and the local index of a cell
struct Omega {
    int64_t ex0 = 0, ey0 = 0, ez0 = 0, EX = 0, EY = 0, EZ = 0;
    std::vector<int64_t> cells;
    std::vector<int32_t> owned;
    std::vector<int32_t> lmap;
    int32_t at(int64_t i, int64_t j, int64_t k) const
    {
        if (i < ex0 || i >= ex0 + EX || j < ey0 || j >= ey0 + EY || k < ez0 || k >= ez0 + EZ) return -1;
        return lmap[((k - ez0) * EY + (j - ey0)) * EX + (i - ex0)];
    }
};

Omega omega_of(const Geo &G, int s, int px, int py, int pz, int ov)
{
    const int64_t nx = G.nx, ny = G.ny, nz = G.nz;
    auto dist = [](int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo - v : (v >= hi ? v - hi + 1 : 0); };
    Omega o;
    const int64_t sx = s % px, sy = (s / px) % py, sz = s / ((int64_t)px * py);
    const int64_t x0 = kbox_start(sx, nx, px), x1 = kbox_start(sx + 1, nx, px);
    const int64_t y0 = kbox_start(sy, ny, py), y1 = kbox_start(sy + 1, ny, py);
    const int64_t z0 = kbox_start(sz, nz, pz), z1 = kbox_start(sz + 1, nz, pz);
    o.ex0 = std::max<int64_t>(0, x0 - ov);
    o.ey0 = std::max<int64_t>(0, y0 - ov);
    o.ez0 = std::max<int64_t>(0, z0 - ov);
    o.EX = std::min<int64_t>(nx, x1 + ov) - o.ex0;
    o.EY = std::min<int64_t>(ny, y1 + ov) - o.ey0;
    o.EZ = std::min<int64_t>(nz, z1 + ov) - o.ez0;
    o.lmap.assign((size_t)(o.EX * o.EY * o.EZ), -1);
    for (int64_t k = o.ez0; k < o.ez0 + o.EZ; ++k)
        for (int64_t j = o.ey0; j < o.ey0 + o.EY; ++j)
            for (int64_t i = o.ex0; i < o.ex0 + o.EX; ++i) {
                if (dist(i, x0, x1) + dist(j, y0, y1) + dist(k, z0, z1) > ov) continue;
                o.lmap[((k - o.ez0) * o.EY + (j - o.ey0)) * o.EX + (i - o.ex0)] = (int32_t)o.cells.size();
                o.cells.push_back((k * ny + j) * nx + i);
                o.owned.push_back(i >= x0 && i < x1 && j >= y0 && j < y1 && k >= z0 && k < z1);
            }
    return o;
}

// symbolic ILU(k) of one subdomain's local matrix, rows in local order
struct SubPlan {
    std::vector<int64_t> cells;                  // global natural cell index, ascending
    std::vector<int32_t> owned;
    std::vector<int64_t> lptr, uptr;             // per local row: its range in lcol / ucol (m + 1)
    std::vector<int32_t> lcol, ucol;             // local columns, ascending within a row
    std::vector<int32_t> flev, blev;
    int nfl = 0, nbl = 0;
};

// Runs f(s) for s = 0 .. n-1 on up to 16 host threads.
template <class F> void for_each_subdomain(int n, F f)
{
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
        th.emplace_back([&, t] { for (int s = t; s < n; s += nth) f(s); });
    for (auto &x : th) x.join();
}

struct RasK final : PcImpl {
    rsv_matrix *M = nullptr;
    rsv_ctx *c = nullptr;
    int nsub = 0;
    int nfl_max = 0, nbl_max = 0;   // most levels of a subdomain (forward, backward)
    bool per_level = false;         // apply by per-level launches
    int64_t nrow = 0, nl = 0, nu = 0;
    std::vector<void *> mem;
    IlukDev d{};

    ~RasK() override
    {
        if (c) (void)hipStreamSynchronize(c->stream);
        for (void *p : mem) dev_free(p);
    }
    int64_t bytes() const override { return (nl + nu) * (72 + 12) + nrow * (2 * 72 + 24 + 32); }
    // per factor block its values and column (76 B); per row the pivot
    // inverse, ids and ranges (120 B), r in, y out, y in, y out, z out (120 B)
    int64_t apply_bytes() const override { return (nl + nu) * 76 + nrow * 240; }

    template <class T> rsv_status upload(T **dp, const std::vector<T> &h)
    {
        rsv_status s = dev_alloc(c, (void **)dp, std::max<size_t>(h.size(), 1) * sizeof(T));
        if (s != RSV_OK) return s;
        mem.push_back(*dp);
        if (!h.empty()) RSV_HIP(c, hipMemcpyAsync(*dp, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
        return RSV_OK;
    }
    template <class T> rsv_status alloc(T **dp, size_t n)
    {
        rsv_status s = dev_alloc(c, (void **)dp, std::max<size_t>(n, 1) * sizeof(T));
        if (s == RSV_OK) mem.push_back(*dp);
        return s;
    }

    rsv_status apply(const double *r, double *z) override
    {
        ProfScope ps(c, RSV_K_RAS);
        return iluk_apply(c, d, nsub, nfl_max, nbl_max, per_level, r, z);
    }

    rsv_status setup(int px, int py, int pz, int ov, int level, int64_t *bad_cell)
    {
        const Geo &G = M->g->geo;
        const int64_t nx = G.nx, ny = G.ny;
        nsub = px * py * pz;
        std::vector<SubPlan> P(nsub);
        auto plan = [&](int s) {
            SubPlan &sp = P[s];
            Omega om = omega_of(G, s, px, py, pz, ov);
            sp.cells = std::move(om.cells);
            sp.owned = std::move(om.owned);
            const int64_t m = (int64_t)sp.cells.size();
            auto at = [&](int64_t i, int64_t j, int64_t k) -> int32_t { return om.at(i, j, k); };
            // rows in order, appended to flat arrays; ulev holds each U entry's fill level
            sp.lptr.assign(m + 1, 0);
            sp.uptr.assign(m + 1, 0);
            std::vector<int32_t> ulev;
            std::vector<int32_t> lev(m, -1), row;
            for (int64_t r = 0; r < m; ++r) {
                const int64_t cc = sp.cells[r];
                const int64_t i = cc % nx, j = (cc / nx) % ny, k = cc / (nx * ny);
                row.clear();
                const int32_t nb[7] = {at(i, j, k - 1), at(i, j - 1, k), at(i - 1, j, k), (int32_t)r,
                                       at(i + 1, j, k), at(i, j + 1, k), at(i, j, k + 1)};
                for (int q = 0; q < 7; ++q)
                    if (nb[q] >= 0) { row.push_back(nb[q]); lev[nb[q]] = 0; }
                std::sort(row.begin(), row.end());
                for (size_t t = 0; t < row.size() && row[t] < r; ++t) {
                    const int32_t mm = row[t];
                    for (int64_t q = sp.uptr[mm]; q < sp.uptr[mm + 1]; ++q) {
                        const int32_t jj = sp.ucol[q];
                        const int32_t l = lev[mm] + ulev[q] + 1;
                        if (l > level) continue;
                        if (lev[jj] < 0) {
                            row.insert(std::upper_bound(row.begin() + t + 1, row.end(), jj), jj);
                            lev[jj] = l;
                        } else if (l < lev[jj]) {
                            lev[jj] = l;
                        }
                    }
                }
                for (int32_t col : row) {
                    if (col < r) sp.lcol.push_back(col);
                    else if (col > r) { sp.ucol.push_back(col); ulev.push_back(lev[col]); }
                    lev[col] = -1;
                }
                sp.lptr[r + 1] = (int64_t)sp.lcol.size();
                sp.uptr[r + 1] = (int64_t)sp.ucol.size();
            }
            sp.flev.assign(m, 0);
            sp.blev.assign(m, 0);
            for (int64_t r = 0; r < m; ++r) {
                int32_t v = 0;
                for (int64_t q = sp.lptr[r]; q < sp.lptr[r + 1]; ++q) v = std::max(v, sp.flev[sp.lcol[q]] + 1);
                sp.flev[r] = v;
                sp.nfl = std::max(sp.nfl, v + 1);
            }
            for (int64_t r = m - 1; r >= 0; --r) {
                int32_t v = 0;
                for (int64_t q = sp.uptr[r]; q < sp.uptr[r + 1]; ++q) v = std::max(v, sp.blev[sp.ucol[q]] + 1);
                sp.blev[r] = v;
                sp.nbl = std::max(sp.nbl, v + 1);
            }
        };
        for_each_subdomain(nsub, plan);
        // concatenate: rows of subdomain s start at base[s]
        std::vector<int64_t> base(nsub + 1, 0);
        for (int s = 0; s < nsub; ++s) base[s + 1] = base[s] + (int64_t)P[s].cells.size();
        nrow = base[nsub];
        if (nrow >= ((int64_t)1 << 31)) return set_err(c, RSV_ERR_ARG, "RAS: more than 2^31 subdomain cells");
        // per subdomain: its first L / U entry and its first level boundary
        std::vector<int64_t> lbase(nsub + 1, 0), ubase(nsub + 1, 0), fbase(nsub + 1, 0), bbase(nsub + 1, 0);
        for (int s = 0; s < nsub; ++s) {
            lbase[s + 1] = lbase[s] + (int64_t)P[s].lcol.size();
            ubase[s + 1] = ubase[s] + (int64_t)P[s].ucol.size();
            fbase[s + 1] = fbase[s] + P[s].nfl + 1;
            bbase[s + 1] = bbase[s] + P[s].nbl + 1;
            nfl_max = std::max(nfl_max, P[s].nfl);
            nbl_max = std::max(nbl_max, P[s].nbl);
        }
        nl = lbase[nsub];
        nu = ubase[nsub];
        std::vector<int32_t> gslot(nrow), own(nrow), lcol(nl), ucol(nu), fo(nrow), bo(nrow);
        std::vector<int64_t> lptr(nrow + 1), uptr(nrow + 1), lsrc(nl), usrc(nu), dbase(nrow), fl(fbase[nsub]),
            bl(bbase[nsub]);
        std::vector<int32_t> fl_off(nsub), bl_off(nsub), fl_cnt(nsub), bl_cnt(nsub);
        auto abase = [&](int64_t cell, int slotdir) -> int64_t {   // A entry of block (cell, stencil slot) at element 0
            const int i = (int)(cell % nx), j = (int)((cell / nx) % ny), k = (int)(cell / (nx * ny));
            return aidx(slot_of(G, i, j, k), slotdir * 9);
        };
        // stencil slot of the position (cell a, column cell b), or -1 for a fill position
        auto stencil_dir = [&](int64_t a, int64_t b) -> int {
            const int64_t di = b % nx - a % nx, dj = (b / nx) % ny - (a / nx) % ny, dk = b / (nx * ny) - a / (nx * ny);
            if (di == 0 && dj == 0 && dk == -1) return 0;
            if (di == 0 && dj == -1 && dk == 0) return 1;
            if (di == -1 && dj == 0 && dk == 0) return 2;
            if (di == 1 && dj == 0 && dk == 0) return 4;
            if (di == 0 && dj == 1 && dk == 0) return 5;
            if (di == 0 && dj == 0 && dk == 1) return 6;
            return -1;
        };
        for_each_subdomain(nsub, [&](int s) {
            const SubPlan &sp = P[s];
            const int64_t m = (int64_t)sp.cells.size();
            for (int64_t r = 0; r < m; ++r) {
                const int64_t g = base[s] + r, cc = sp.cells[r];
                const int i = (int)(cc % nx), j = (int)((cc / nx) % ny), k = (int)(cc / (nx * ny));
                gslot[g] = (int32_t)slot_of(G, i, j, k);
                // the owner bit, and the cell's row for error reports
                own[g] = (int32_t)((row_of(G, i, j, k) << 1) | (sp.owned[r] ? 1 : 0));
                dbase[g] = abase(cc, 3);
                lptr[g] = lbase[s] + sp.lptr[r];
                for (int64_t q = sp.lptr[r]; q < sp.lptr[r + 1]; ++q) {
                    const int32_t col = sp.lcol[q];
                    lcol[lbase[s] + q] = (int32_t)(base[s] + col);
                    const int dir = stencil_dir(cc, sp.cells[col]);
                    lsrc[lbase[s] + q] = dir >= 0 ? abase(cc, dir) : -1;
                }
                uptr[g] = ubase[s] + sp.uptr[r];
                for (int64_t q = sp.uptr[r]; q < sp.uptr[r + 1]; ++q) {
                    const int32_t col = sp.ucol[q];
                    ucol[ubase[s] + q] = (int32_t)(base[s] + col);
                    const int dir = stencil_dir(cc, sp.cells[col]);
                    usrc[ubase[s] + q] = dir >= 0 ? abase(cc, dir) : -1;
                }
            }
            // level schedules: the subdomain's rows bucketed by level
            for (int pass = 0; pass < 2; ++pass) {
                const std::vector<int32_t> &lv = pass ? sp.blev : sp.flev;
                const int nlv = pass ? sp.nbl : sp.nfl;
                std::vector<int64_t> cnt(nlv + 1, 0);
                for (int64_t r = 0; r < m; ++r) cnt[lv[r] + 1]++;
                for (int q = 0; q < nlv; ++q) cnt[q + 1] += cnt[q];
                const int64_t b0 = pass ? bbase[s] : fbase[s];
                (pass ? bl_off : fl_off)[s] = (int32_t)b0;
                (pass ? bl_cnt : fl_cnt)[s] = nlv;
                std::vector<int64_t> &bounds = pass ? bl : fl;
                for (int q = 0; q <= nlv; ++q) bounds[b0 + q] = base[s] + cnt[q];
                std::vector<int32_t> &ord = pass ? bo : fo;
                std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
                for (int64_t r = 0; r < m; ++r) ord[base[s] + fill[lv[r]]++] = (int32_t)(base[s] + r);
            }
        });
        lptr[nrow] = nl;
        uptr[nrow] = nu;
        P.clear();
        per_level = nsub > 0 && nrow / nsub >= 256 * (int64_t)std::max(nfl_max, nbl_max);
        int32_t *dgslot, *down, *dlcol, *ducol, *dfo, *dbo, *dfloff, *dbloff, *dflcnt, *dblcnt;
        int64_t *dlptr, *duptr, *dlsrc, *dusrc, *ddbase, *dfl, *dbl;
        double *dlval, *duval, *ddval, *ddinv, *dy;
        rsv_status st = upload(&dgslot, gslot);
        if (st == RSV_OK) st = upload(&down, own);
        if (st == RSV_OK) st = upload(&dlptr, lptr);
        if (st == RSV_OK) st = upload(&duptr, uptr);
        if (st == RSV_OK) st = upload(&dlcol, lcol);
        if (st == RSV_OK) st = upload(&ducol, ucol);
        if (st == RSV_OK) st = upload(&dlsrc, lsrc);
        if (st == RSV_OK) st = upload(&dusrc, usrc);
        if (st == RSV_OK) st = upload(&ddbase, dbase);
        if (st == RSV_OK) st = upload(&dfo, fo);
        if (st == RSV_OK) st = upload(&dbo, bo);
        if (st == RSV_OK) st = upload(&dfl, fl);
        if (st == RSV_OK) st = upload(&dbl, bl);
        if (st == RSV_OK) st = upload(&dfloff, fl_off);
        if (st == RSV_OK) st = upload(&dbloff, bl_off);
        if (st == RSV_OK) st = upload(&dflcnt, fl_cnt);
        if (st == RSV_OK) st = upload(&dblcnt, bl_cnt);
        if (st == RSV_OK) st = alloc(&dlval, (size_t)9 * nl);
        if (st == RSV_OK) st = alloc(&duval, (size_t)9 * nu);
        if (st == RSV_OK) st = alloc(&ddval, (size_t)9 * nrow);
        if (st == RSV_OK) st = alloc(&ddinv, (size_t)9 * nrow);
        if (st == RSV_OK) st = alloc(&dy, (size_t)3 * nrow);
        if (st != RSV_OK) return st;
        d = IlukDev{nrow, dgslot, down, dlptr, duptr, dlptr + 1, duptr + 1, dlcol, ducol, dlsrc, dusrc, dlval, duval,
                    ddval, ddinv, dy, dfo, dbo, dfl, dbl, dfloff, dbloff, dflcnt, dblcnt, ddbase};
        rsv_status fs = flags_reset(c);      // synchronises: the host arrays may go after this
        if (fs != RSV_OK) return fs;
        {
            ProfScope ps(c, RSV_K_FACTOR);
            const int64_t tot = nl + nu + nrow;
            hipLaunchKernelGGL(k_iluk_load, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, M->d_A, d,
                               nl, nu);
            hipLaunchKernelGGL(k_iluk_factor, dim3(nsub), dim3(KT), 0, c->stream, d, c->d_flags);
        }
        RSV_LAUNCH(c);
        return flags_check(c, bad_cell);
    }
};

// ILUT(p, tol) local solvers: the host lays out Omega_s and the local
// stencil (value-independent), the device factors and schedules
struct RasT final : PcImpl {
    rsv_matrix *M = nullptr;
    rsv_ctx *c = nullptr;
    int nsub = 0;
    int nfl_max = 0, nbl_max = 0;   // most levels of a subdomain (forward, backward)
    bool per_level = false;         // apply by per-level launches
    int64_t nrow = 0, capl = 0, capu = 0;
    std::vector<void *> mem;
    IlukDev d{};

    ~RasT() override
    {
        if (c) (void)hipStreamSynchronize(c->stream);
        for (void *p : mem) dev_free(p);
    }
    int64_t bytes() const override { return nrow * ((capl + capu) * 76 + 2 * 72 + 24 + 7 * 12 + 48); }
    int64_t nkept = 0;            // factor blocks kept (L and U, diagonals apart)
    int64_t apply_bytes() const override { return nkept * 76 + nrow * 240; }

    template <class T> rsv_status upload(T **dp, const std::vector<T> &h)
    {
        rsv_status s = dev_alloc(c, (void **)dp, std::max<size_t>(h.size(), 1) * sizeof(T));
        if (s != RSV_OK) return s;
        mem.push_back(*dp);
        if (!h.empty()) RSV_HIP(c, hipMemcpyAsync(*dp, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
        return RSV_OK;
    }
    template <class T> rsv_status alloc(T **dp, size_t n)
    {
        rsv_status s = dev_alloc(c, (void **)dp, std::max<size_t>(n, 1) * sizeof(T));
        if (s == RSV_OK) mem.push_back(*dp);
        return s;
    }

    rsv_status apply(const double *r, double *z) override
    {
        ProfScope ps(c, RSV_K_RAS);
        return iluk_apply(c, d, nsub, nfl_max, nbl_max, per_level, r, z);
    }

    rsv_status setup(int px, int py, int pz, int ov, int p, double tol, int64_t *bad_cell)
    {
        const Geo &G = M->g->geo;
        const int64_t nx = G.nx, ny = G.ny;
        nsub = px * py * pz;
        capl = capu = (p < 0) ? 3 : p;
        std::vector<Omega> O(nsub);
        for_each_subdomain(nsub, [&](int s) { O[s] = omega_of(G, s, px, py, pz, ov); });
        std::vector<int64_t> base(nsub + 1, 0);
        for (int s = 0; s < nsub; ++s) base[s + 1] = base[s] + (int64_t)O[s].cells.size();
        nrow = base[nsub];
        if (nrow >= ((int64_t)1 << 31)) return set_err(c, RSV_ERR_ARG, "ILUT: more than 2^31 subdomain cells");
        std::vector<int32_t> gslot(nrow), own(nrow), acol(7 * nrow, -1), subw(nsub), floff(nsub);
        std::vector<int64_t> asrc(7 * nrow, -1), lptr(nrow), uptr(nrow);
        const size_t lds_fixed = (size_t)T_NBUF * (9 * 8 + 8 + 4 + 4 + 1 + 1) + (size_t)(T_LCAP + T_CAP_MAX) * 4;
        for (int s = 0; s < nsub; ++s) {
            const Omega &om = O[s];
            const int64_t m = (int64_t)om.cells.size();
            int64_t bw = 0;
            for (int64_t r = 0; r < m; ++r) {
                const int64_t g = base[s] + r, cc = om.cells[r];
                const int i = (int)(cc % nx), j = (int)((cc / nx) % ny), k = (int)(cc / (nx * ny));
                gslot[g] = (int32_t)slot_of(G, i, j, k);
                own[g] = (int32_t)((row_of(G, i, j, k) << 1) | (om.owned[r] ? 1 : 0));
                lptr[g] = g * capl;
                uptr[g] = g * capu;
                const int32_t nb[7] = {om.at(i, j, k - 1), om.at(i, j - 1, k), om.at(i - 1, j, k), (int32_t)r,
                                       om.at(i + 1, j, k), om.at(i, j + 1, k), om.at(i, j, k + 1)};
                // block (row, direction st) sits at the row's own slot
                const int64_t rs = slot_of(G, i, j, k);
                for (int st = 0; st < 7; ++st) {
                    if (nb[st] < 0) continue;
                    acol[7 * g + st] = (int32_t)(base[s] + nb[st]);
                    bw = std::max<int64_t>(bw, std::abs((int64_t)nb[st] - r));
                    asrc[7 * g + st] = aidx(rs, st * 9);
                }
            }
            subw[s] = (int32_t)(2 * bw + 1);
            floff[s] = (int32_t)(base[s] + s);
            if (lds_fixed + 2 * (size_t)subw[s] + 1024 > (size_t)c->lds_max)   // 1 KiB for the static LDS
                return set_err(c, RSV_ERR_ARG, "ILUT: a subdomain's band is too wide for the work row in LDS; use more RAS subdomains");
        }
        size_t lds = lds_fixed + 2 * (size_t)*std::max_element(subw.begin(), subw.end());
        O.clear();
        int32_t *dgslot, *down, *dacol, *dsubw, *dfloff, *dlcol, *ducol, *dflev, *dblev, *dfo, *dbo, *dflcnt, *dblcnt;
        int64_t *dasrc, *dbase, *dlptr, *duptr, *dlend, *duend, *dfl, *dbl, *dcnt, *dnk;
        double *dlval, *duval, *ddval, *ddinv, *dy;
        rsv_status st = upload(&dgslot, gslot);
        if (st == RSV_OK) st = upload(&down, own);
        if (st == RSV_OK) st = upload(&dacol, acol);
        if (st == RSV_OK) st = upload(&dasrc, asrc);
        if (st == RSV_OK) st = upload(&dbase, base);
        if (st == RSV_OK) st = upload(&dsubw, subw);
        if (st == RSV_OK) st = upload(&dfloff, floff);
        if (st == RSV_OK) st = upload(&dlptr, lptr);
        if (st == RSV_OK) st = upload(&duptr, uptr);
        if (st == RSV_OK) st = alloc(&dlend, (size_t)nrow);
        if (st == RSV_OK) st = alloc(&duend, (size_t)nrow);
        if (st == RSV_OK) st = alloc(&dlcol, (size_t)(nrow * capl));
        if (st == RSV_OK) st = alloc(&ducol, (size_t)(nrow * capu));
        if (st == RSV_OK) st = alloc(&dlval, (size_t)(9 * nrow * capl));
        if (st == RSV_OK) st = alloc(&duval, (size_t)(9 * nrow * capu));
        if (st == RSV_OK) st = alloc(&ddval, (size_t)(9 * nrow));
        if (st == RSV_OK) st = alloc(&ddinv, (size_t)(9 * nrow));
        if (st == RSV_OK) st = alloc(&dy, (size_t)(3 * nrow));
        if (st == RSV_OK) st = alloc(&dflev, (size_t)nrow);
        if (st == RSV_OK) st = alloc(&dblev, (size_t)nrow);
        if (st == RSV_OK) st = alloc(&dfo, (size_t)nrow);
        if (st == RSV_OK) st = alloc(&dbo, (size_t)nrow);
        if (st == RSV_OK) st = alloc(&dfl, (size_t)(nrow + nsub));
        if (st == RSV_OK) st = alloc(&dbl, (size_t)(nrow + nsub));
        if (st == RSV_OK) st = alloc(&dcnt, (size_t)(nrow + nsub));
        if (st == RSV_OK) st = alloc(&dflcnt, (size_t)nsub);
        if (st == RSV_OK) st = alloc(&dblcnt, (size_t)nsub);
        if (st == RSV_OK) st = alloc(&dnk, (size_t)nsub);
        if (st != RSV_OK) return st;
        IlutDev t{nrow, dacol, dasrc, dbase, dsubw, down, p, (int32_t)capl, (int32_t)capu, tol * tol, dlptr, duptr,
                  dlend, duend, dlcol, ducol, dlval, duval, ddval, ddinv, dflev, dblev, dfo, dbo, dfl, dbl, dflcnt,
                  dblcnt, dcnt, dnk};
        d = IlukDev{nrow, dgslot, down, dlptr, duptr, dlend, duend, dlcol, ducol, nullptr, nullptr, dlval, duval,
                    ddval, ddinv, dy, dfo, dbo, dfl, dbl, dfloff, dfloff, dflcnt, dblcnt, nullptr};
        rsv_status fs = flags_reset(c);      // synchronises: the host arrays may go after this
        if (fs != RSV_OK) return fs;
        if (lds > 65536)
            RSV_HIP(c, hipFuncSetAttribute((const void *)k_ilut_factor, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds));
        {
            ProfScope ps(c, RSV_K_FACTOR);
            hipLaunchKernelGGL(k_ilut_factor, dim3(nsub), dim3(TW), lds, c->stream, t, (const double *)M->d_A,
                               c->d_flags);
        }
        RSV_LAUNCH(c);
        int32_t f[2];
        RSV_HIP(c, hipMemcpyAsync(f, c->d_flags, sizeof(f), hipMemcpyDeviceToHost, c->stream));
        RSV_HIP(c, hipStreamSynchronize(c->stream));
        if (f[0] & FLAG_ILUT_CAP)
            return set_err(c, RSV_ERR_ARG, "ILUT: a row's work list outgrew its 512 blocks; raise ilut_tol or set ilut_p");
        rsv_status fc = flags_check(c, bad_cell);
        if (fc != RSV_OK) return fc;
        std::vector<int64_t> nk(nsub);
        RSV_HIP(c, hipMemcpy(nk.data(), dnk, (size_t)nsub * sizeof(int64_t), hipMemcpyDeviceToHost));
        nkept = 0;
        for (int64_t v : nk) nkept += v;
        // the device-built schedules' level counts choose the apply
        std::vector<int32_t> nfc(nsub), nbc(nsub);
        RSV_HIP(c, hipMemcpy(nfc.data(), d.fl_cnt, (size_t)nsub * sizeof(int32_t), hipMemcpyDeviceToHost));
        RSV_HIP(c, hipMemcpy(nbc.data(), d.bl_cnt, (size_t)nsub * sizeof(int32_t), hipMemcpyDeviceToHost));
        nfl_max = *std::max_element(nfc.begin(), nfc.end());
        nbl_max = *std::max_element(nbc.begin(), nbc.end());
        per_level = nrow / nsub >= 256 * (int64_t)std::max(nfl_max, nbl_max);
        return RSV_OK;
    }
};

}  // namespace

rsv_status rasK_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell)
{
    rsv_ctx *c = A->g->ctx;
    const Geo &G = A->g->geo;
    int px = 1, py = 1, pz = 1, ov = 0;      // BILU(k) of the whole grid: one subdomain, no overlap
    if (p->type == RSV_PC_RAS) {
        px = p->ras_px; py = p->ras_py; pz = p->ras_pz; ov = p->ras_overlap;
        if (px < 1 || py < 1 || pz < 1 || px > G.nx || py > G.ny || pz > G.nz || ov < 0)
            return set_err(c, RSV_ERR_ARG, "bad RAS subdomain counts or overlap");
    }
    if (p->precision != RSV_FP64) return set_err(c, RSV_ERR_ARG, "ILU(k) with k > 0 has FP64 factors only");
    if (p->iluk_level < 1 || p->iluk_level > 8) return set_err(c, RSV_ERR_ARG, "iluk_level must be in [0, 8]");
    RasK *R = new (std::nothrow) RasK();
    if (!R) return set_err(c, RSV_ERR_OOM, "ILU(k) RAS");
    R->M = A;
    R->c = c;
    rsv_status s = R->setup(px, py, pz, ov, p->iluk_level, bad_cell);
    if (s != RSV_OK) {
        delete R;
        return s;
    }
    *out = R;
    return RSV_OK;
}

rsv_status rasT_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell)
{
    rsv_ctx *c = A->g->ctx;
    const Geo &G = A->g->geo;
    int px = 1, py = 1, pz = 1, ov = 0;      // ILUT of the whole grid: one subdomain, no overlap
    if (p->type == RSV_PC_RAS) {
        px = p->ras_px; py = p->ras_py; pz = p->ras_pz; ov = p->ras_overlap;
        if (px < 1 || py < 1 || pz < 1 || px > G.nx || py > G.ny || pz > G.nz || ov < 0)
            return set_err(c, RSV_ERR_ARG, "bad RAS subdomain counts or overlap");
    }
    if (p->precision != RSV_FP64) return set_err(c, RSV_ERR_ARG, "ILUT has FP64 factors only");
    if (p->ilut_p < -1 || p->ilut_p > T_CAP_MAX) return set_err(c, RSV_ERR_ARG, "ilut_p must be in [-1, 32]");
    if (!(p->ilut_tol >= 0.0) || !std::isfinite(p->ilut_tol)) return set_err(c, RSV_ERR_ARG, "ilut_tol must be >= 0");
    RasT *R = new (std::nothrow) RasT();
    if (!R) return set_err(c, RSV_ERR_OOM, "ILUT RAS");
    R->M = A;
    R->c = c;
    rsv_status s = R->setup(px, py, pz, ov, p->ilut_p, p->ilut_tol, bad_cell);
    if (s != RSV_OK) {
        delete R;
        return s;
    }
    *out = R;
    return RSV_OK;
}
