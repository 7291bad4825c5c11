// Block ILU(0) of the 7-point, 3x3-block matrix in natural (bottom-up) order:
// factorisation and the two triangular sweeps (Preconditioners section: LU x
// = b <=> L y = b, U x = y, solved row by row; ILU(0) is the default local
// solver of the RAS default-parameter figure).
//
// On the bipartite 7-point graph, ILU(0) reduces to pivots
//   D_c = A_cc - sum_{k in {-z,-y,-x}} A_ck D_k^{-1} A_kc,
// with L_ck = A_ck D_k^{-1} (unit lower factor) and U = D + strict upper of A.
// Cell c depends only on its -x,-y,-z neighbours, all on hyperplane
// i+j+k-1, so processing hyperplanes in order reproduces natural-order ILU(0)
// exactly (same operations per cell; only the FP order inside a cell may
// differ from a row-by-row code).
//
// Two executions of the sweeps:
//  * one launch per hyperplane (reference; also the factorisation);
//  * a pipelined tile-lane kernel: each wavefront owns an 8x8 column of cells,
//    lane (i,j) walks up the column skewed by i+j steps, lanes exchange the
//    previous step's values by cross-lane shuffles, and neighbouring tiles
//    hand over their boundary faces through epoch-tagged 64-bit words (value
//    and tag in one single-copy-atomic word, so no fences are needed).  Tiles
//    are taken from an atomic ticket in topological order, so a tile only
//    ever waits on tiles already held by running wavefronts (no deadlock);
//    every wait is bounded by a wall-clock limit that raises an error flag.
#include "rsv_internal.h"

#include <algorithm>
#include <new>

namespace {

constexpr int BS = 256;
constexpr uint64_t SPIN_LIMIT_TICKS = 200000000ull;   // 2 s of the 100 MHz wall clock

__device__ inline int64_t fidx(int64_t slot, int e, int ne) { return ((slot >> 6) * ne + e) * 64 + (slot & 63); }

// Per-cell arithmetic shared by the per-hyperplane and the pipelined sweeps,
// so that both executions produce bitwise-identical results.
// forward: out = r - (L_-z vz + L_-y vy + L_-x vx)   (ascending column order)
template <typename T>
__device__ __forceinline__ void fwd_cell(const T *l, const T *vz, const T *vy, const T *vx, const T *rr, T *out)
{
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        T acc = l[3 * p] * vz[0] + l[3 * p + 1] * vz[1] + l[3 * p + 2] * vz[2];
        acc += l[9 + 3 * p] * vy[0] + l[9 + 3 * p + 1] * vy[1] + l[9 + 3 * p + 2] * vy[2];
        acc += l[18 + 3 * p] * vx[0] + l[18 + 3 * p + 1] * vx[1] + l[18 + 3 * p + 2] * vx[2];
        out[p] = rr[p] - acc;
    }
}
// backward: out = Dinv (y - (U_+x vx + U_+y vy + U_+z vz))
template <typename T>
__device__ __forceinline__ void bwd_cell(const T *u, const T *dd, const T *vx, const T *vy, const T *vz, const T *yy,
                                         T *out)
{
    T tv[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        T acc = u[3 * p] * vx[0] + u[3 * p + 1] * vx[1] + u[3 * p + 2] * vx[2];
        acc += u[9 + 3 * p] * vy[0] + u[9 + 3 * p + 1] * vy[1] + u[9 + 3 * p + 2] * vy[2];
        acc += u[18 + 3 * p] * vz[0] + u[18 + 3 * p + 1] * vz[1] + u[18 + 3 * p + 2] * vz[2];
        tv[p] = yy[p] - acc;
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) out[p] = dd[3 * p] * tv[0] + dd[3 * p + 1] * tv[1] + dd[3 * p + 2] * tv[2];
}

// ---------------------------------------------------------------- factorisation (one launch per hyperplane)
__global__ __launch_bounds__(BS) void k_factor_plane(Geo g, const int32_t *__restrict__ slots, int64_t n,
                                                     const double *__restrict__ A, double *__restrict__ Lf,
                                                     double *__restrict__ Dinv, int32_t *flags)
{
    const int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (t >= n) return;
    const int64_t slot = slots[t];
    int gx, gy, k;
    cell_of(g, slot, gx, gy, k);
    double D[9];
    for (int e = 0; e < 9; ++e) D[e] = A[aidx(slot, 27 + e)];
    for (int s = 0; s < 3; ++s) {   // -z, -y, -x: ascending column order
        int di, dj, dk;
        dir_off(s, di, dj, dk);
        double L[9];
        if (gx + di >= 0 && gy + dj >= 0 && k + dk >= 0) {
            const int64_t ns = slot_of(g, gx + di, gy + dj, k + dk);
            double Ack[9], Dk[9], Akc[9];
            for (int e = 0; e < 9; ++e) {
                Ack[e] = A[aidx(slot, s * 9 + e)];
                Dk[e] = Dinv[fidx(ns, e, 9)];
                Akc[e] = A[aidx(ns, (6 - s) * 9 + e)];
            }
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q)
                    L[3 * p + q] = Ack[3 * p] * Dk[q] + Ack[3 * p + 1] * Dk[3 + q] + Ack[3 * p + 2] * Dk[6 + q];
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q)
                    D[3 * p + q] -= L[3 * p] * Akc[q] + L[3 * p + 1] * Akc[3 + q] + L[3 * p + 2] * Akc[6 + q];
        } else {
            for (int e = 0; e < 9; ++e) L[e] = 0.0;
        }
        for (int e = 0; e < 9; ++e) Lf[fidx(slot, s * 9 + e, 27)] = L[e];
    }
    double Di[9];
    if (!inv3(D, Di)) {
        atomicOr(&flags[0], FLAG_PIVOT);
        atomicMin(&flags[1], (int32_t)row_of(g, gx, gy, k));
        for (int e = 0; e < 9; ++e) Di[e] = 0.0;
    }
    for (int e = 0; e < 9; ++e) Dinv[fidx(slot, e, 9)] = Di[e];
}

template <typename T>
__global__ __launch_bounds__(BS) void k_to_f32(int64_t n, const double *__restrict__ a, T *__restrict__ b)
{
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS) b[e] = (T)a[e];
}

// strict upper blocks of A (+x,+y,+z) as FP32 in [row][27][64]
__global__ __launch_bounds__(BS) void k_upper_f32(int64_t nslot, const double *__restrict__ A, float *__restrict__ U)
{
    const int64_t slot = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (slot >= nslot) return;
    for (int e = 0; e < 27; ++e) U[fidx(slot, e, 27)] = (float)A[aidx(slot, 36 + e)];
}

// ---------------------------------------------------------------- sweeps, one launch per hyperplane
// T: arithmetic / factor type.  Upper blocks: U (T, [row][27][64]) when
// non-null, else the FP64 matrix A directly.
template <typename T>
__global__ __launch_bounds__(BS) void k_fwd_plane(Geo g, const int32_t *__restrict__ slots, int64_t n,
                                                  const T *__restrict__ Lf, const double *__restrict__ r,
                                                  T *__restrict__ y)
{
    const int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (t >= n) return;
    const int64_t slot = slots[t];
    int gx, gy, k;
    cell_of(g, slot, gx, gy, k);
    T v[3][3];   // -z, -y, -x neighbour values
    for (int s = 0; s < 3; ++s) {
        int di, dj, dk;
        dir_off(s, di, dj, dk);
        v[s][0] = v[s][1] = v[s][2] = 0;
        if (gx + di >= 0 && gy + dj >= 0 && k + dk >= 0) {
            const int64_t ns = slot_of(g, gx + di, gy + dj, k + dk);
            for (int p = 0; p < 3; ++p) v[s][p] = y[vidx(ns, p)];
        }
    }
    T l[27], rr[3], out[3];
    for (int e = 0; e < 27; ++e) l[e] = Lf[fidx(slot, e, 27)];
    for (int p = 0; p < 3; ++p) rr[p] = (T)r[vidx(slot, p)];
    fwd_cell(l, v[0], v[1], v[2], rr, out);
    for (int p = 0; p < 3; ++p) y[vidx(slot, p)] = out[p];
}

template <typename T>
__global__ __launch_bounds__(BS) void k_bwd_plane(Geo g, const int32_t *__restrict__ slots, int64_t n,
                                                  const T *__restrict__ Dinv, const T *__restrict__ U,
                                                  const double *__restrict__ A, const T *__restrict__ y,
                                                  T *__restrict__ zt, double *__restrict__ z)
{
    const int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (t >= n) return;
    const int64_t slot = slots[t];
    int gx, gy, k;
    cell_of(g, slot, gx, gy, k);
    T v[3][3];   // +x, +y, +z neighbour values
    for (int s = 4; s < 7; ++s) {
        int di, dj, dk;
        dir_off(s, di, dj, dk);
        v[s - 4][0] = v[s - 4][1] = v[s - 4][2] = 0;
        if (gx + di < g.nx && gy + dj < g.ny && k + dk < g.nz) {
            const int64_t ns = slot_of(g, gx + di, gy + dj, k + dk);
            for (int p = 0; p < 3; ++p) v[s - 4][p] = zt[vidx(ns, p)];
        }
    }
    T u[27], dd[9], yy[3], out[3];
    for (int e = 0; e < 27; ++e) u[e] = U ? U[fidx(slot, e, 27)] : (T)A[aidx(slot, 36 + e)];
    for (int e = 0; e < 9; ++e) dd[e] = Dinv[fidx(slot, e, 9)];
    for (int p = 0; p < 3; ++p) yy[p] = y[vidx(slot, p)];
    bwd_cell(u, dd, v[0], v[1], v[2], yy, out);
    for (int p = 0; p < 3; ++p) {
        zt[vidx(slot, p)] = out[p];
        z[vidx(slot, p)] = (double)out[p];
    }
}

// ---------------------------------------------------------------- pipelined tile-lane sweeps

// Face words: FP64 values are split into two 32-bit halves, each stored with
// the 32-bit epoch in the upper half of a 64-bit word; FP32 values take one word.
template <typename T> struct FaceW;
template <> struct FaceW<double> { static constexpr int W = 2; };
template <> struct FaceW<float> { static constexpr int W = 1; };

__device__ inline void face_put(uint64_t *p, double v, uint32_t ep)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    __hip_atomic_store(p, ((uint64_t)ep << 32) | (b & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, ((uint64_t)ep << 32) | (b >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void face_put(uint64_t *p, float v, uint32_t ep)
{
    __hip_atomic_store(p, ((uint64_t)ep << 32) | (uint64_t)__float_as_uint(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t face_ld(const uint64_t *p)
{
    return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double face_val(const uint64_t *w, double) { return __longlong_as_double((long long)((w[0] & 0xffffffffull) | (w[1] << 32))); }
__device__ inline float face_val(const uint64_t *w, float) { return __uint_as_float((uint32_t)w[0]); }

template <typename T>
struct FaceSet {
    uint64_t w[3 * FaceW<T>::W];
};

template <typename T>
__device__ inline void face_load3(FaceSet<T> &f, const uint64_t *p)
{
#pragma unroll
    for (int q = 0; q < 3 * FaceW<T>::W; ++q) f.w[q] = face_ld(p + q);
}

template <typename T>
__device__ inline bool face_ok(const FaceSet<T> &f, uint32_t ep)
{
    bool ok = true;
#pragma unroll
    for (int q = 0; q < 3 * FaceW<T>::W; ++q) ok = ok && ((uint32_t)(f.w[q] >> 32) == ep);
    return ok;
}

// Wait (bounded) until the three values at p carry epoch ep; returns them.
template <typename T>
__device__ inline void face_wait(FaceSet<T> &f, const uint64_t *p, uint32_t ep, int32_t *flags, T *out)
{
    if (!face_ok(f, ep)) {
        const uint64_t t0 = wall_clock64();
        for (;;) {
            face_load3(f, p);
            if (face_ok(f, ep)) break;
            // give up at the bound, or at once if another wait already timed out
            const int32_t fl = __hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((fl & FLAG_TIMEOUT) || wall_clock64() - t0 > SPIN_LIMIT_TICKS) {
                atomicOr(&flags[0], FLAG_TIMEOUT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    const int W = FaceW<T>::W;
#pragma unroll
    for (int p3 = 0; p3 < 3; ++p3) out[p3] = face_val(&f.w[p3 * W], T());
}

__device__ inline double shfl_d(double v, int src) { return __shfl(v, src, 64); }
__device__ inline float shfl_d(float v, int src) { return __shfl(v, src, 64); }

struct SweepArgs {
    Geo g;
    const int32_t *tile_order;   // tiles in topological (anti-diagonal) order
    uint64_t *ticket;
    uint64_t ticket_base;
    uint64_t *faceX;             // [NT][nz][8][3][W]
    uint64_t *faceY;
    uint32_t epoch;
    int32_t *flags;
};

// Forward sweep y = L^{-1} r.  NE = 27 factor entries per cell.
template <typename T, int PD>
__global__ __launch_bounds__(64) void k_sweep_fwd(SweepArgs a, const T *__restrict__ Lf,
                                                 const double *__restrict__ r, T *__restrict__ y)
{
    constexpr int W = FaceW<T>::W;
    const Geo &g = a.g;
    const int L = threadIdx.x;
    int li, lj;
    lane_ij(L, li, lj);
    const int d = li + lj;
    const int lx = (li > 0) ? ij_lane(li - 1, lj) : L;
    const int ly = (lj > 0) ? ij_lane(li, lj - 1) : L;
    const int NT = g.ntx * g.nty;
    const int nz = g.nz;
    const int nsteps = nz + 14;
    for (;;) {
        uint64_t tk = 0;
        if (L == 0) tk = atomicAdd((unsigned long long *)a.ticket, 1ull);
        tk = __shfl(tk, 0, 64) - a.ticket_base;
        if (tk >= (uint64_t)NT) break;
        const int T_ = a.tile_order[tk];
        const int tx = T_ % g.ntx, ty = T_ / g.ntx;
        const int64_t rowbase = (int64_t)T_ * nz;
        const bool cx = (li == 0 && tx > 0), cy = (lj == 0 && ty > 0);
        const bool px = (li == 7 && tx < g.ntx - 1), py = (lj == 7 && ty < g.nty - 1);
        const uint64_t *fxin = a.faceX + ((int64_t)(T_ - 1) * nz * 8 * 3 * W);
        const uint64_t *fyin = a.faceY + ((int64_t)(T_ - g.ntx) * nz * 8 * 3 * W);
        uint64_t *fxout = a.faceX + ((int64_t)T_ * nz * 8 * 3 * W);
        uint64_t *fyout = a.faceY + ((int64_t)T_ * nz * 8 * 3 * W);

        T ring_l[PD][27];
        double ring_r[PD][3];
        FaceSet<T> ring_fx[PD], ring_fy[PD];
        auto issue = [&](int u, int t) {
            const int k = t - d;
            if (t < nsteps && k >= 0 && k < nz) {
                const int row = wrap_nz(t, nz);
                const T *lp = Lf + ((rowbase + row) * 27) * 64 + L;
#pragma unroll
                for (int e = 0; e < 27; ++e) ring_l[u][e] = lp[e * 64];
                const double *rp = r + (rowbase + row) * 192 + L;
#pragma unroll
                for (int p = 0; p < 3; ++p) ring_r[u][p] = rp[p * 64];
                if (cx) face_load3(ring_fx[u], fxin + ((int64_t)k * 8 + lj) * 3 * W);
                if (cy) face_load3(ring_fy[u], fyin + ((int64_t)k * 8 + li) * 3 * W);
            }
        };
#pragma unroll
        for (int u = 0; u < PD; ++u) issue(u, u);
        T last[3] = {0, 0, 0};
        for (int t0 = 0; t0 < nsteps; t0 += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                const int t = t0 + u;
                if (t < nsteps) {
                    const int k = t - d;
                    const bool act = (k >= 0 && k < nz);
                    T vx[3], vy[3], vz[3];
#pragma unroll
                    for (int p = 0; p < 3; ++p) {
                        vx[p] = shfl_d(last[p], lx);
                        vy[p] = shfl_d(last[p], ly);
                        vz[p] = last[p];
                    }
                    T out[3] = {0, 0, 0};
                    if (act) {
                        if (li == 0) {
                            if (cx) face_wait(ring_fx[u], fxin + ((int64_t)k * 8 + lj) * 3 * W, a.epoch, a.flags, vx);
                            else vx[0] = vx[1] = vx[2] = 0;
                        }
                        if (lj == 0) {
                            if (cy) face_wait(ring_fy[u], fyin + ((int64_t)k * 8 + li) * 3 * W, a.epoch, a.flags, vy);
                            else vy[0] = vy[1] = vy[2] = 0;
                        }
                        if (k == 0) vz[0] = vz[1] = vz[2] = 0;
                        T rr[3] = {(T)ring_r[u][0], (T)ring_r[u][1], (T)ring_r[u][2]};
                        fwd_cell(ring_l[u], vz, vy, vx, rr, out);
                        const int row = wrap_nz(t, nz);
                        T *yp = y + (rowbase + row) * 192 + L;
#pragma unroll
                        for (int p = 0; p < 3; ++p) yp[p * 64] = out[p];
                        if (px) {
                            uint64_t *f = fxout + ((int64_t)k * 8 + lj) * 3 * W;
#pragma unroll
                            for (int p = 0; p < 3; ++p) face_put(f + p * W, out[p], a.epoch);
                        }
                        if (py) {
                            uint64_t *f = fyout + ((int64_t)k * 8 + li) * 3 * W;
#pragma unroll
                            for (int p = 0; p < 3; ++p) face_put(f + p * W, out[p], a.epoch);
                        }
                    }
#pragma unroll
                    for (int p = 0; p < 3; ++p) last[p] = out[p];
                    issue(u, t + PD);
                }
            }
        }
    }
}

// Backward sweep z = U^{-1} y.  Upper blocks are read at U + row*u_stride +
// u_off: the FP32 copy [row][27][64], or the FP64 matrix A itself (offset 36*64).
template <typename T, int PD>
__global__ __launch_bounds__(64) void k_sweep_bwd(SweepArgs a, const T *__restrict__ Dinv,
                                                 const T *__restrict__ U, int64_t u_stride, int64_t u_off,
                                                 const T *__restrict__ y, double *__restrict__ z)
{
    constexpr int W = FaceW<T>::W;
    const Geo &g = a.g;
    const int L = threadIdx.x;
    int li, lj;
    lane_ij(L, li, lj);
    const int e_ = 14 - (li + lj);
    const int lx = (li < 7) ? ij_lane(li + 1, lj) : L;
    const int ly = (lj < 7) ? ij_lane(li, lj + 1) : L;
    const int NT = g.ntx * g.nty;
    const int nz = g.nz;
    const int nsteps = nz + 14;
    for (;;) {
        uint64_t tk = 0;
        if (L == 0) tk = atomicAdd((unsigned long long *)a.ticket, 1ull);
        tk = __shfl(tk, 0, 64) - a.ticket_base;
        if (tk >= (uint64_t)NT) break;
        const int T_ = a.tile_order[NT - 1 - (int)tk];
        const int tx = T_ % g.ntx, ty = T_ / g.ntx;
        const int64_t rowbase = (int64_t)T_ * nz;
        const bool cx = (li == 7 && tx < g.ntx - 1), cy = (lj == 7 && ty < g.nty - 1);
        const bool px = (li == 0 && tx > 0), py = (lj == 0 && ty > 0);
        const uint64_t *fxin = a.faceX + ((int64_t)(T_ + 1) * nz * 8 * 3 * W);
        const uint64_t *fyin = a.faceY + ((int64_t)(T_ + g.ntx) * nz * 8 * 3 * W);
        uint64_t *fxout = a.faceX + ((int64_t)T_ * nz * 8 * 3 * W);
        uint64_t *fyout = a.faceY + ((int64_t)T_ * nz * 8 * 3 * W);

        T ring_u[PD][27];
        T ring_d[PD][9];
        T ring_y[PD][3];
        FaceSet<T> ring_fx[PD], ring_fy[PD];
        auto issue = [&](int u, int t) {
            const int kk = t - e_;
            if (t < nsteps && kk >= 0 && kk < nz) {
                const int k = nz - 1 - kk;
                const int row = wrap_nz(nz + 13 - t, nz);
                const T *up = U + (rowbase + row) * u_stride + u_off + L;
#pragma unroll
                for (int e = 0; e < 27; ++e) ring_u[u][e] = up[e * 64];
                const T *dp = Dinv + ((rowbase + row) * 9) * 64 + L;
#pragma unroll
                for (int e = 0; e < 9; ++e) ring_d[u][e] = dp[e * 64];
                const T *yp = y + (rowbase + row) * 192 + L;
#pragma unroll
                for (int p = 0; p < 3; ++p) ring_y[u][p] = yp[p * 64];
                if (cx) face_load3(ring_fx[u], fxin + ((int64_t)k * 8 + lj) * 3 * W);
                if (cy) face_load3(ring_fy[u], fyin + ((int64_t)k * 8 + li) * 3 * W);
            }
        };
#pragma unroll
        for (int u = 0; u < PD; ++u) issue(u, u);
        T last[3] = {0, 0, 0};
        for (int t0 = 0; t0 < nsteps; t0 += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                const int t = t0 + u;
                if (t < nsteps) {
                    const int kk = t - e_;
                    const bool act = (kk >= 0 && kk < nz);
                    const int k = nz - 1 - kk;
                    T vx[3], vy[3], vz[3];
#pragma unroll
                    for (int p = 0; p < 3; ++p) {
                        vx[p] = shfl_d(last[p], lx);
                        vy[p] = shfl_d(last[p], ly);
                        vz[p] = last[p];
                    }
                    T out[3] = {0, 0, 0};
                    if (act) {
                        if (li == 7) {
                            if (cx) face_wait(ring_fx[u], fxin + ((int64_t)k * 8 + lj) * 3 * W, a.epoch, a.flags, vx);
                            else vx[0] = vx[1] = vx[2] = 0;
                        }
                        if (lj == 7) {
                            if (cy) face_wait(ring_fy[u], fyin + ((int64_t)k * 8 + li) * 3 * W, a.epoch, a.flags, vy);
                            else vy[0] = vy[1] = vy[2] = 0;
                        }
                        if (kk == 0) vz[0] = vz[1] = vz[2] = 0;
                        bwd_cell(ring_u[u], ring_d[u], vx, vy, vz, ring_y[u], out);
                        const int row = wrap_nz(nz + 13 - t, nz);
                        double *zp = z + (rowbase + row) * 192 + L;
#pragma unroll
                        for (int p = 0; p < 3; ++p) zp[p * 64] = (double)out[p];
                        if (px) {
                            uint64_t *f = fxout + ((int64_t)k * 8 + lj) * 3 * W;
#pragma unroll
                            for (int p = 0; p < 3; ++p) face_put(f + p * W, out[p], a.epoch);
                        }
                        if (py) {
                            uint64_t *f = fyout + ((int64_t)k * 8 + li) * 3 * W;
#pragma unroll
                            for (int p = 0; p < 3; ++p) face_put(f + p * W, out[p], a.epoch);
                        }
                    }
#pragma unroll
                    for (int p = 0; p < 3; ++p) last[p] = out[p];
                    issue(u, t + PD);
                }
            }
        }
    }
}

// ---------------------------------------------------------------- the preconditioner object

struct Bilu0 : PcImpl {
    rsv_matrix *M = nullptr;
    rsv_ctx *c = nullptr;
    bool fp32 = false;
    bool pipelined = true;
    double *Lf = nullptr, *Dinv = nullptr;      // FP64 factors [row][27|9][64]
    float *Lf32 = nullptr, *Dinv32 = nullptr, *U32 = nullptr;
    void *ybuf = nullptr;                        // T-typed intermediate vector
    float *zt32 = nullptr;                       // FP32 z for the per-plane path
    double *zt64 = nullptr;
    uint64_t *faceX = nullptr, *faceY = nullptr;
    int32_t *tile_order = nullptr;
    int64_t nbytes = 0;

    ~Bilu0() override
    {
        dev_free(Lf); dev_free(Dinv); dev_free(Lf32); dev_free(Dinv32); dev_free(U32);
        dev_free(ybuf); dev_free(zt32); dev_free(zt64); dev_free(faceX); dev_free(faceY); dev_free(tile_order);
    }
    int64_t bytes() const override { return nbytes; }

    rsv_status alloc(void **p, size_t b)
    {
        rsv_status s = dev_alloc(c, p, b);
        if (s == RSV_OK) {
            nbytes += (int64_t)b;
            hipError_t e = hipMemsetAsync(*p, 0, b, c->stream);
            if (e != hipSuccess) return set_err(c, RSV_ERR_HIP, "hipMemsetAsync");
        }
        return s;
    }

    rsv_status setup(int64_t *bad_cell)
    {
        const Geo &g = M->g->geo;
        const int64_t rows = g.nslot / 64;
        rsv_status s = alloc((void **)&Lf, (size_t)rows * 27 * 64 * sizeof(double));
        if (s == RSV_OK) s = alloc((void **)&Dinv, (size_t)rows * 9 * 64 * sizeof(double));
        if (s != RSV_OK) return s;
        s = flags_reset(c);
        if (s != RSV_OK) return s;
        ProfScope ps(c, RSV_K_FACTOR);
        for (int p = 0; p < M->g->nplanes; ++p) {
            const int64_t off = M->g->plane_ptr[p], n = M->g->plane_ptr[p + 1] - off;
            if (n == 0) continue;
            hipLaunchKernelGGL(k_factor_plane, dim3((unsigned)((n + BS - 1) / BS)), dim3(BS), 0, c->stream, g,
                               M->g->d_plane_slots + off, n, M->d_A, Lf, Dinv, c->d_flags);
            RSV_LAUNCH(c);
        }
        s = flags_check(c, bad_cell);
        if (s != RSV_OK) return s;
        const int NT = g.ntx * g.nty;
        if (fp32) {
            s = alloc((void **)&Lf32, (size_t)rows * 27 * 64 * sizeof(float));
            if (s == RSV_OK) s = alloc((void **)&Dinv32, (size_t)rows * 9 * 64 * sizeof(float));
            if (s == RSV_OK) s = alloc((void **)&U32, (size_t)rows * 27 * 64 * sizeof(float));
            if (s == RSV_OK) s = alloc(&ybuf, (size_t)M->g->nv * sizeof(float));
            if (s == RSV_OK) s = alloc((void **)&zt32, (size_t)M->g->nv * sizeof(float));
            if (s != RSV_OK) return s;
            hipLaunchKernelGGL(k_to_f32<float>, dim3(2048), dim3(BS), 0, c->stream, rows * 27 * 64, Lf, Lf32);
            hipLaunchKernelGGL(k_to_f32<float>, dim3(2048), dim3(BS), 0, c->stream, rows * 9 * 64, Dinv, Dinv32);
            hipLaunchKernelGGL(k_upper_f32, dim3((unsigned)((g.nslot + BS - 1) / BS)), dim3(BS), 0, c->stream,
                               g.nslot, M->d_A, U32);
            RSV_LAUNCH(c);
            // FP64 factors are not needed by the FP32 sweeps
            RSV_HIP(c, hipStreamSynchronize(c->stream));
            dev_free(Lf); Lf = nullptr;
            dev_free(Dinv); Dinv = nullptr;
            nbytes -= (int64_t)rows * 36 * 64 * sizeof(double);
        } else {
            s = alloc(&ybuf, (size_t)M->g->nv * sizeof(double));
            if (s == RSV_OK) s = alloc((void **)&zt64, (size_t)M->g->nv * sizeof(double));
            if (s != RSV_OK) return s;
        }
        if (pipelined) {
            const int W = fp32 ? 1 : 2;
            const size_t fb = (size_t)NT * g.nz * 8 * 3 * W * sizeof(uint64_t);
            s = alloc((void **)&faceX, fb);
            if (s == RSV_OK) s = alloc((void **)&faceY, fb);
            if (s == RSV_OK) s = alloc((void **)&tile_order, (size_t)NT * sizeof(int32_t));
            if (s != RSV_OK) return s;
            std::vector<int32_t> ord(NT);
            for (int t = 0; t < NT; ++t) ord[t] = t;
            std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
                const int da = a % g.ntx + a / g.ntx, db = b % g.ntx + b / g.ntx;
                return da < db;
            });
            RSV_HIP(c, hipMemcpy(tile_order, ord.data(), NT * sizeof(int32_t), hipMemcpyHostToDevice));
        }
        RSV_HIP(c, hipStreamSynchronize(c->stream));
        return RSV_OK;
    }

    template <typename T>
    rsv_status apply_plane(const double *r, double *z, const T *L_, const T *D_, const T *U_, T *zt)
    {
        const Geo &g = M->g->geo;
        T *y = (T *)ybuf;
        for (int p = 0; p < M->g->nplanes; ++p) {
            const int64_t off = M->g->plane_ptr[p], n = M->g->plane_ptr[p + 1] - off;
            if (n == 0) continue;
            hipLaunchKernelGGL(k_fwd_plane<T>, dim3((unsigned)((n + BS - 1) / BS)), dim3(BS), 0, c->stream, g,
                               M->g->d_plane_slots + off, n, L_, r, y);
        }
        RSV_LAUNCH(c);
        for (int p = M->g->nplanes - 1; p >= 0; --p) {
            const int64_t off = M->g->plane_ptr[p], n = M->g->plane_ptr[p + 1] - off;
            if (n == 0) continue;
            hipLaunchKernelGGL(k_bwd_plane<T>, dim3((unsigned)((n + BS - 1) / BS)), dim3(BS), 0, c->stream, g,
                               M->g->d_plane_slots + off, n, D_, U_, M->d_A, (const T *)y, zt, z);
        }
        RSV_LAUNCH(c);
        return RSV_OK;
    }

    SweepArgs sweep_args(uint64_t nwaves)
    {
        const Geo &g = M->g->geo;
        SweepArgs a;
        a.g = g;
        a.tile_order = tile_order;
        a.ticket = c->d_tickets;
        a.ticket_base = c->ticket_base[0];
        a.faceX = faceX;
        a.faceY = faceY;
        a.epoch = c->epoch++;
        if (c->epoch == 0) c->epoch = 1;
        a.flags = c->d_flags;
        c->ticket_base[0] += (uint64_t)(g.ntx * g.nty) + nwaves;
        return a;
    }

    int nwaves() const
    {
        const int NT = M->g->geo.ntx * M->g->geo.nty;
        return std::max(1, std::min(NT, c->num_cu * 4));
    }

    rsv_status apply(const double *r, double *z) override
    {
        if (!pipelined) {
            ProfScope ps(c, RSV_K_ILU_FWD);
            if (fp32) return apply_plane<float>(r, z, Lf32, Dinv32, U32, zt32);
            return apply_plane<double>(r, z, Lf, Dinv, nullptr, zt64);
        }
        const int nw = nwaves();
        if (fp32) {
            SweepArgs a = sweep_args(nw);
            int t1 = prof_begin(c, RSV_K_ILU_FWD);
            hipLaunchKernelGGL((k_sweep_fwd<float, 4>), dim3(nw), dim3(64), 0, c->stream, a, Lf32, r, (float *)ybuf);
            prof_end(c, t1);
            RSV_LAUNCH(c);
            SweepArgs b = sweep_args(nw);
            int t2 = prof_begin(c, RSV_K_ILU_BWD);
            hipLaunchKernelGGL((k_sweep_bwd<float, 4>), dim3(nw), dim3(64), 0, c->stream, b, Dinv32, U32,
                               (int64_t)27 * 64, (int64_t)0, (const float *)ybuf, z);
            prof_end(c, t2);
            RSV_LAUNCH(c);
        } else {
            SweepArgs a = sweep_args(nw);
            int t1 = prof_begin(c, RSV_K_ILU_FWD);
            hipLaunchKernelGGL((k_sweep_fwd<double, 3>), dim3(nw), dim3(64), 0, c->stream, a, Lf, r, (double *)ybuf);
            prof_end(c, t1);
            RSV_LAUNCH(c);
            SweepArgs b = sweep_args(nw);
            int t2 = prof_begin(c, RSV_K_ILU_BWD);
            hipLaunchKernelGGL((k_sweep_bwd<double, 3>), dim3(nw), dim3(64), 0, c->stream, b, Dinv, M->d_A,
                               (int64_t)63 * 64, (int64_t)36 * 64, (const double *)ybuf, z);
            prof_end(c, t2);
            RSV_LAUNCH(c);
        }
        return RSV_OK;
    }
};

}  // namespace

rsv_status bilu0_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell)
{
    rsv_ctx *c = A->g->ctx;
    Bilu0 *B = new (std::nothrow) Bilu0();
    if (!B) return set_err(c, RSV_ERR_OOM, "bilu0");
    B->M = A;
    B->c = c;
    B->fp32 = (p->precision == RSV_FP32);
    B->pipelined = (p->pipelined != 0);
    rsv_status s = B->setup(bad_cell);
    if (s != RSV_OK) {
        delete B;
        return s;
    }
    *out = B;
    return RSV_OK;
}
