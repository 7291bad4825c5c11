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
#include <cstdio>
#include <cstdlib>
#include <new>

namespace {

constexpr int BS = 256;

__device__ inline int64_t fidx(int64_t slot, int e, int ne) { return ((slot >> 6) * ne + e) * 64 + (slot & 63); }

// Per-cell arithmetic shared by the per-hyperplane and the pipelined sweeps,
// so that both executions produce bitwise-identical results.
// forward: out = r - (L_-z vz + L_-y vy + L_-x vx)   (ascending column order)
// explicit fused multiply-adds: the same operation sequence in every kernel
// that inlines these helpers, whatever the contraction choices around them
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// forward: out = r - (L_-z vz + L_-y vy + L_-x vx), one FMA chain per
// component (terms in the order -z, -y, -x), the three chains advanced in
// lockstep; negated products are free operand modifiers
template <typename T>
__device__ __forceinline__ void fwd_cell(const T *l, const T *vz, const T *vy, const T *vx, const T *rr, T *out)
{
    T acc[3] = {rr[0], rr[1], rr[2]};
    const T *v[3] = {vz, vy, vx};
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int p = 0; p < 3; ++p) acc[p] = fma_t(-l[9 * s + 3 * p + q], v[s][q], acc[p]);
#pragma unroll
    for (int p = 0; p < 3; ++p) out[p] = acc[p];
}
// backward: out = Dinv (y - (U_+x vx + U_+y vy + U_+z vz)), same chain order (+x, +y, +z)
template <typename T>
__device__ __forceinline__ void bwd_cell(const T *u, const T *dd, const T *vx, const T *vy, const T *vz, const T *yy,
                                         T *out)
{
    T tv[3] = {yy[0], yy[1], yy[2]};
    const T *v[3] = {vx, vy, vz};
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int p = 0; p < 3; ++p) tv[p] = fma_t(-u[9 * s + 3 * p + q], v[s][q], tv[p]);
#pragma unroll
    for (int p = 0; p < 3; ++p) out[p] = fma_t(dd[3 * p + 2], tv[2], fma_t(dd[3 * p + 1], tv[1], dd[3 * p] * tv[0]));
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

// factors of the real slots into block-row order: L[row][27], Dinv[row][9]
__global__ __launch_bounds__(BS) void k_factors_to_rows(Geo g, const double *__restrict__ Lf,
                                                        const double *__restrict__ Dinv, double *__restrict__ Lr,
                                                        double *__restrict__ Dr)
{
    const int64_t slot = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (slot >= g.nslot) return;
    int gx, gy, k;
    if (!cell_of(g, slot, gx, gy, k)) return;
    const int64_t row = row_of(g, gx, gy, k);
    for (int e = 0; e < 27; ++e) Lr[row * 27 + e] = Lf[fidx(slot, e, 27)];
    for (int e = 0; e < 9; ++e) Dr[row * 9 + e] = Dinv[fidx(slot, e, 9)];
}

// ---------------------------------------------------------------- pipelined tile-lane sweeps
//
// One workgroup per tile at a time: wave 0 computes, waves 1..NL stream the
// tile's per-step data into a ring of D slots in LDS (warp specialisation).
// A wavefront can keep at most 63 memory operations outstanding and retires
// them in order, so one wave alone cannot hide HBM latency for the ~30 loads
// each step needs; each loader wave owns every NL-th step and brings its own
// outstanding-load budget.  The compute wave leaves each step's results in
// the step's slot; the loader that refills the slot D steps later first
// stores them to HBM.  A wave's memory instructions queue behind the loads
// of the CU's other waves, so every store the compute wave issued itself
// would hold up its chain of steps (measured: 25 % of the sweep time on
// tiles without neighbours); it stores only the face rows.
//
// Step t of a tile: lane (i,j) of the compute wave handles cell k = t - (i+j)
// (forward) or k = nz-1-(t-(14-i-j)) (backward); the cell's data sit in row
// (t mod nz) (forward) or ((nz+13-t) mod nz) (backward) of the tile, so every
// load is one coalesced 64-lane row.
//
// Face exchange between neighbouring tiles: face row s of a tile holds the
// eight boundary values (three components each) that the neighbouring tile
// needs at its local step s; the producing lane computes them at its own step
// s + 7.  FP64 values are split into 32-bit halves, each stored with the
// 32-bit call epoch in the upper half of a 64-bit word (FP32 values: one
// word), so a word is valid exactly when its tag equals the current epoch --
// no fences between tiles, no clearing between calls (the buffers are cleared
// once, when allocated: memory another object wrote, possibly under another
// context's epochs, could otherwise hold a word with a matching tag).  Word (p*W + h)*8 + e
// of a row holds half h of component p of entry e.  The compute wave writes
// a whole face row with one store instruction (for the same reason, the
// number of store instructions, not their width, sets their cost): lane q
// takes word q of the row from the results in LDS, where the boundary lane
// has just put them.  The loader of step t
// reads the row (one word per lane), waits until every needed word carries
// the epoch, and writes the values into the slot.  Tiles are handed out by an
// atomic ticket in topological order, so a tile only waits on tiles held by
// running workgroups; every wait is bounded by a wall-clock limit that raises
// an error flag and makes all other waits give up at once.

template <typename T> struct FaceW;
template <> struct FaceW<double> { static constexpr int W = 2; };
template <> struct FaceW<float> { static constexpr int W = 1; };

__device__ inline uint64_t face_ld(const uint64_t *p)
{
    return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void face_st(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 32-bit half h of a value's bits (h = 0 for FP32)
__device__ inline uint32_t half_bits(double v, int h) { return (uint32_t)((uint64_t)__double_as_longlong(v) >> (32 * h)); }
__device__ inline uint32_t half_bits(float v, int) { return __float_as_uint(v); }

// Spin-loop guard: checks the clock and the shared error flag only every 256th
// call (the flag read is a device-scope load, which waits for every memory
// operation the wave still has in flight).
__device__ inline bool spin_guard(int32_t *flags, uint64_t t0, uint32_t &n, uint64_t limit)
{
    if ((++n & 255u) != 0u) return false;
    const int32_t fl = __hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (fl & FLAG_TIMEOUT) return true;
    if (wall_clock64() - t0 > limit) {
        atomicOr(&flags[0], FLAG_TIMEOUT);
        return true;
    }
    return false;
}


struct SweepArgs {
    Geo g;
    const int32_t *tile_order;   // tiles in topological (anti-diagonal) order
    uint64_t *ticket;
    uint64_t ticket_base;
    uint64_t *faceX;             // [NT][nz+7][24*W] words
    uint64_t *faceY;
    uint32_t epoch;
    int32_t *flags;
    uint64_t wait_limit;         // wall-clock ticks a wait may last
    int D;                       // LDS ring slots
    int btx, bty;                // tiles per box in x and y: faces are exchanged only between
                                 // tiles of one box (the whole grid is one box for BILU0)
    uint64_t *trace;             // optional: per tile [start, step 8 reached, end, steps that waited for data]
};

// per-step operands streamed by the loaders; all rows are [entries][64 lanes]
template <typename T>
struct SweepSrc {
    const T *p0; int64_t s0, o0;                  // factor blocks (27): L (fwd) or U (bwd)
    const T *p1; int64_t s1, o1;                  // D^{-1} (bwd only, 9)
    const double *v64; const T *vT;               // 3-vector input: r (FP64, fwd) or y (T, bwd)
    const int32_t *zmap;                          // bwd, optional: slot of the output vector that takes
                                                  // each cell's result ([slot], -1: no store); null:
                                                  // the output has this grid's layout
};

// NLOAD loader waves per workgroup (each keeps two steps in flight)
template <int DIR, typename T, int NLOAD>
__global__ __launch_bounds__(64 * (1 + NLOAD)) void k_sweep(SweepArgs a, SweepSrc<T> src, T *__restrict__ yout,
                                                           double *__restrict__ zout)
{
    constexpr int W = FaceW<T>::W;
    constexpr int RW = 24 * W;                   // face words per row
    extern __shared__ __align__(16) unsigned char smem[];
    const Geo &g = a.g;
    const int nz = g.nz, NT = g.ntx * g.nty, nsteps = nz + 14;
    const int D = a.D;
    constexpr int NE = DIR == 0 ? 30 : 39;       // T entries per lane per step (27 blocks [+9 D^-1] + 3 vector)
    constexpr int NS = DIR == 0 ? NE : NE + 1;   // + the output map entry (bwd)
    constexpr int RES = NS * 64 + 48;            // + x and y faces (8 entries x 3 components each)
    constexpr int slot_elems = RES + 192;        // + the step's results ([64 lanes][3])
    T *ring = (T *)smem;
    int32_t *tags = (int32_t *)(smem + (size_t)D * slot_elems * sizeof(T));
    int32_t *consumed = tags + D;
    int32_t *tile_ring = consumed + 1;   // tile of the workgroup's k-th tile in entry k mod 4
    int32_t *tile_tag = tile_ring + 4;   // k + 1 once entry k mod 4 holds the k-th tile
    int32_t *ftags = tile_tag + 4;       // per slot: step whose face values are in the slot (+1)
    const int wave = threadIdx.x >> 6, L = threadIdx.x & 63;
    int li, lj;
    lane_ij(L, li, lj);
    const int64_t frow = (int64_t)(nz + 7) * RW;
    // Tiles come from an atomic ticket (-1 past the last tile).  The k-th tile
    // of this workgroup is published by the first loader wave when it has
    // issued its last step of tile k - 1 (so tiles are still claimed close to
    // when a workgroup can take them up), and the loaders stream the next
    // tile's first steps while the compute wave finishes the current one;
    // there is no barrier between tiles.  Four entries: an entry is rewritten only after
    // every wave has read it (no wave is more than one tile behind another,
    // since the loaders run at most D < nsteps steps ahead of the compute wave).
    auto take = [&]() -> int32_t {
        const uint64_t tk = atomicAdd((unsigned long long *)a.ticket, 1ull) - a.ticket_base;
        return (tk >= (uint64_t)NT) ? -1 : a.tile_order[DIR == 0 ? (int)tk : NT - 1 - (int)tk];
    };
    auto publish = [&](int k) {
        const int32_t id = take();
        __hip_atomic_store(&tile_ring[k & 3], id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __hip_atomic_store(&tile_tag[k & 3], k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    if (threadIdx.x == 0) *consumed = 0;
    for (int s = threadIdx.x; s < D; s += blockDim.x) tags[s] = ftags[s] = 0;
    if (threadIdx.x < 4) tile_tag[threadIdx.x] = 0;
    __syncthreads();
    if (threadIdx.x == 0) publish(0);
    __syncthreads();
    int gstep = 0;   // running step count across tiles (tags are gstep + 1)
    int prevT = -1;  // the workgroup's previous tile
    bool aborted = false;
    // Loader part: the results of global step Gs (tile Ts, local step ts),
    // which the compute wave left in slot sl, go to HBM (lanes whose cell is
    // in range).  The loader that refills a slot does this first, so the
    // compute wave issues no stores of its own besides the face rows.
    auto store_results = [&](const T *sl, int Ts, int ts) {
        const int kk = DIR == 0 ? ts - (li + lj) : ts - (14 - li - lj);
        if (Ts < 0 || kk < 0 || kk >= nz) return;
        const T *res = sl + RES + L * 3;
        const int row = DIR == 0 ? wrap_nz(ts, nz) : wrap_nz(nz + 13 - ts, nz);
        const int64_t rb = (int64_t)Ts * nz + row;
        if constexpr (DIR == 0) {
            T *yp = yout + rb * 192 + L;
#pragma unroll
            for (int p = 0; p < 3; ++p) __builtin_nontemporal_store(res[p], yp + p * 64);
        } else {
            int64_t o = rb * 192 + L;
            if (src.zmap) {
                const int32_t zm = ((const int32_t *)(sl + NE * 64))[L];
                if (zm < 0) return;
                o = ((int64_t)zm >> 6) * 192 + (zm & 63);
            }
#pragma unroll
            for (int p = 0; p < 3; ++p) __builtin_nontemporal_store((double)res[p], zout + o + p * 64);
        }
    };
    for (int k = 0;; ++k) {
        if (__hip_atomic_load(&tile_tag[k & 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != k + 1) {
            const uint64_t t0 = wall_clock64();
            uint32_t n = 0;
            bool gave_up = false;
            while (__hip_atomic_load(&tile_tag[k & 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != k + 1) {
                if (spin_guard(a.flags, t0, n, a.wait_limit)) {
                    gave_up = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (gave_up) {   // the error flag is set; every wave leaves
                aborted = true;
                break;
            }
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const int T_ = __hip_atomic_load(&tile_ring[k & 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (T_ < 0) break;
        const int tx = T_ % g.ntx, ty = T_ / g.ntx;
        const int64_t rowbase = (int64_t)T_ * nz;
        const int bx = tx % a.btx, by = ty % a.bty;   // tile position inside its box
        const bool hasx = DIR == 0 ? bx > 0 : bx < a.btx - 1;
        const bool hasy = DIR == 0 ? by > 0 : by < a.bty - 1;
        if (wave > 0) {
            // ------------------------------------------------ loader waves
            const uint64_t *xin = a.faceX + (int64_t)(DIR == 0 ? T_ - 1 : T_ + 1) * frow;
            const uint64_t *yin = a.faceY + (int64_t)(DIR == 0 ? T_ - g.ntx : T_ + g.ntx) * frow;
            const int eq = L & 7;                    // face entry of this lane's word
            const int fdst = (eq * 3 + (L >> 3) / W) * W + (L >> 3) % W;   // its 32-bit half in the slot's [8][3] values
            constexpr int nv = DIR == 0 ? 27 : 36;
            struct Regs {
                T v[nv + 3];
                int32_t zm;        // output map entry (bwd with a map)
                uint64_t wx, wy;   // face words of the same step
            };
            // face words: always two loads per lane (a tile without that neighbour
            // reads its own face buffer, an in-range dummy); validity is decided later
            const uint64_t *xsrc = hasx ? xin : a.faceX + (int64_t)T_ * frow;
            const uint64_t *ysrc = hasy ? yin : a.faceY + (int64_t)T_ * frow;
            const int lq = L < RW ? L : RW - 1;
            // loads are issued unconditionally (out-of-range steps re-read a valid
            // row) so that the outstanding-load count is static and the compiler
            // can wait for exactly the buffer it needs
            // Lanes are ordered by anti-diagonal, so the lanes whose cell is in range
            // at step t are one contiguous range [lo, hi]; an out-of-range lane reads
            // the slot of the nearest in-range lane instead of its own, so a step
            // touches only the cache lines its in-range lanes need (the wrapped
            // layout would otherwise re-read rows at the start and end of a column).
            auto issue_lane = [&](int tc) {
                const int dmin = DIR == 0 ? (tc - nz + 1 > 0 ? tc - nz + 1 : 0) : (14 - tc > 0 ? 14 - tc : 0);
                const int dmax = DIR == 0 ? (tc < 14 ? tc : 14) : (13 - tc + nz < 14 ? 13 - tc + nz : 14);
                const int lo = lane_first(dmin), hi = lane_first(dmax + 1) - 1;
                return L < lo ? lo : (L > hi ? hi : L);
            };
            // The factor blocks are read once per apply and the results written
            // once: both bypass the caches' retention (nontemporal; measured
            // 3-4 % faster sweeps on the 512x512x128 grid).
            auto issue_data = [&](Regs &R, int t) {
                const int tc = t < nsteps ? t : nsteps - 1;
                const int row = DIR == 0 ? wrap_nz(tc, nz) : wrap_nz(nz + 13 - tc, nz);
                const int64_t rb = rowbase + row;
                const int Ls = issue_lane(tc);
                const T *q0 = src.p0 + rb * src.s0 + src.o0 + Ls;
#pragma unroll
                for (int e = 0; e < 27; ++e) R.v[e] = __builtin_nontemporal_load(q0 + e * 64);
                if constexpr (DIR == 1) {
                    const T *q1 = src.p1 + rb * src.s1 + src.o1 + Ls;
#pragma unroll
                    for (int e = 0; e < 9; ++e) R.v[27 + e] = __builtin_nontemporal_load(q1 + e * 64);
                }
                if constexpr (DIR == 0) {
                    const double *q2 = src.v64 + rb * 192 + Ls;
#pragma unroll
                    for (int p = 0; p < 3; ++p) R.v[nv + p] = (T)q2[p * 64];
                } else {
                    const T *q2 = src.vT + rb * 192 + Ls;
#pragma unroll
                    for (int p = 0; p < 3; ++p) R.v[nv + p] = q2[p * 64];
                    R.zm = src.zmap ? src.zmap[rb * 64 + Ls] : -1;
                }
                // face words of the same step, issued with its data (they may still
                // be stale when the step is delivered; then they are polled again)
                const int tr = t < nz + 7 ? t : nz + 6;
                R.wx = face_ld(xsrc + (int64_t)tr * RW + lq);
                R.wy = face_ld(ysrc + (int64_t)tr * RW + lq);
            };
            // face words of step t (entries whose cell exists)
            auto face_need = [&](int t) {
                const int kk = DIR == 0 ? t - eq : t - 7 + eq;
                return L < RW && kk >= 0 && kk < nz;
            };
            auto finish = [&](const Regs &R, int t) {
                uint64_t wx = R.wx, wy = R.wy;
                const int G = gstep + t;
                const int slot = G % D;
                T *sl = ring + (size_t)slot * slot_elems;
                // wait for the compute wave to release this slot (step G - D)
                if (__hip_atomic_load(consumed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < G - D + 1) {
                    const uint64_t t0 = wall_clock64();
                    uint32_t n = 0;
                    while (__hip_atomic_load(consumed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < G - D + 1) {
                        if (spin_guard(a.flags, t0, n, a.wait_limit)) break;
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                // the slot still holds the results of step G - D (this tile's or the previous one's)
                if (G >= D) {
                    const int Gs = G - D;
                    const bool cur = Gs >= gstep;
                    store_results(sl, cur ? T_ : prevT, cur ? Gs - gstep : Gs - gstep + nsteps);
                }
#pragma unroll
                for (int e = 0; e < nv + 3; ++e) sl[e * 64 + L] = R.v[e];
                if constexpr (DIR == 1) ((int32_t *)(sl + NE * 64))[L] = R.zm;
                // operands first (the compute wave prefetches them while faces are pending)
                __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                __hip_atomic_store(&tags[slot], G + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                const bool need = face_need(t);
                const bool okx = !hasx || !need || (uint32_t)(wx >> 32) == a.epoch;
                const bool oky = !hasy || !need || (uint32_t)(wy >> 32) == a.epoch;
                if (!(okx && oky)) {
                    // Slow path.  Seven loaders: every loader polls its own
                    // step's rows at a short fixed interval, so consecutive
                    // steps are not serialised on each other's poll round trips.
                    // Backward FP64 sweep (three loaders): rows become valid in
                    // step order, so first wait (in LDS) until the previous step
                    // has been delivered; then only the loader of the oldest
                    // pending step polls device memory, with exponential backoff
                    // up to four 512-cycle sleeps.  (Measured: the first is
                    // faster forward, the second backward; a cap of 16 sleeps
                    // made the backward sweep at 128x128x64 4 % slower.)
                    const uint64_t t0 = wall_clock64();
                    uint32_t n = 0;
                    constexpr bool serial = NLOAD < 7;
                    if (serial && t > 0)
                        while (__hip_atomic_load(&ftags[(G - 1) % D], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < G) {
                            if (spin_guard(a.flags, t0, n, a.wait_limit)) break;
                            __builtin_amdgcn_s_sleep(2);
                        }
                    int backoff = 1;
                    for (;;) {
                        if (hasx) wx = face_ld(xin + (int64_t)t * RW + lq);
                        if (hasy) wy = face_ld(yin + (int64_t)t * RW + lq);
                        const bool ok = (!hasx || !need || (uint32_t)(wx >> 32) == a.epoch) &&
                                        (!hasy || !need || (uint32_t)(wy >> 32) == a.epoch);
                        if (__ballot(!ok) == 0ull) break;
                        if (spin_guard(a.flags, t0, n, a.wait_limit)) break;
                        if (!serial) {
                            __builtin_amdgcn_s_sleep(2);
                        } else {
                            for (int q = 0; q < backoff; ++q) __builtin_amdgcn_s_sleep(8);
                            backoff = backoff < 4 ? 2 * backoff : 4;
                        }
                    }
                }
                // the low 32 bits of word q are 32-bit half q of the row's values
                // (zero when the tile has no such neighbour: the value of an absent cell)
                uint32_t *fs = (uint32_t *)(sl + NS * 64);
                if (L < RW) {
                    fs[fdst] = hasx ? (uint32_t)wx : 0u;
                    fs[RW + fdst] = hasy ? (uint32_t)wy : 0u;
                }
                // the face writes complete before the face tag is published
                __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                __hip_atomic_store(&ftags[slot], G + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            };
            // two steps in flight per loader: the next step's loads are issued
            // before the current one is delivered
            Regs A, B;
            int t = wave - 1;
            issue_data(A, t);
            for (; t < nsteps; t += 2 * NLOAD) {
                issue_data(B, t + NLOAD);
                finish(A, t);
                if (t + NLOAD >= nsteps) break;
                issue_data(A, t + 2 * NLOAD);
                finish(B, t + NLOAD);
            }
            if (wave == 1 && L == 0) publish(k + 1);
        } else {
            // ------------------------------------------------ compute wave
            const int d = li + lj;
            const int e_ = 14 - d;
            const int lx = DIR == 0 ? (li > 0 ? ij_lane(li - 1, lj) : L) : (li < 7 ? ij_lane(li + 1, lj) : L);
            const int ly = DIR == 0 ? (lj > 0 ? ij_lane(li, lj - 1) : L) : (lj < 7 ? ij_lane(li, lj + 1) : L);
            const bool cx = DIR == 0 ? li == 0 : li == 7, cy = DIR == 0 ? lj == 0 : lj == 7;
            // packed face stores: lane q < RW owns word q of each outgoing face
            // row, half h = (q >> 3) % W of component (q >> 3) / W of entry
            // e = q & 7, read from the result row of the boundary lane of
            // entry e (x face: i = 7 forward, 0 backward, j = e; y face: i = e)
            const int fe = L & 7, fp = (L >> 3) / W, fh = (L >> 3) % W;
            const int fbx = DIR == 0 ? 7 : 0;
            const int fx_src = ij_lane(fbx, fe) * 3 + fp;   // in the step's result rows
            const int fy_src = ij_lane(fe, fbx) * 3 + fp;
            const bool fxw = L < RW && (DIR == 0 ? bx < a.btx - 1 : bx > 0);
            const bool fyw = L < RW && (DIR == 0 ? by < a.bty - 1 : by > 0);
            // the boundary cell of entry e at step t is in range when (t - fk0) is in [0, nz)
            const int fk0 = DIR == 0 ? 7 + fe : 14 - fe;
            uint64_t *fxo = a.faceX + (int64_t)T_ * frow + L;
            uint64_t *fyo = a.faceY + (int64_t)T_ * frow + L;
            uint32_t waited = 0;
            if (a.trace && L == 0) a.trace[4 * T_ + 0] = wall_clock64();
            // Neighbour values come through LDS: every step the wave writes its
            // three results into the result rows of the step's slot; at the next
            // step an interior lane reads the row of its -x (+x) and -y (+y)
            // neighbour lane there (the slot is released for new operands, but
            // its result rows are rewritten only by this wave, D steps later),
            // and a boundary lane reads the face entry the loader put in the
            // step's slot.  One wave only, so its LDS accesses stay in program
            // order.  At a tile's first step the previous slot holds another
            // tile's results, but only the lane of the tile corner is in range
            // then, and it takes both values from faces.
            const uint32_t slot_bytes = (uint32_t)slot_elems * sizeof(T);
            const uint32_t xo_int = (uint32_t)(RES + lx * 3) * sizeof(T);
            const uint32_t yo_int = (uint32_t)(RES + ly * 3) * sizeof(T);
            const uint32_t xo_face = (uint32_t)(NS * 64 + lj * 3) * sizeof(T);
            const uint32_t yo_face = (uint32_t)(NS * 64 + 24 + li * 3) * sizeof(T);
            T last[3] = {0, 0, 0};   // this lane's previous result: the -z (+z) neighbour value
            // spin until the loaders have delivered step G into `slot` (tag G + 1);
            // `seen` is a tag value already read
            auto wait_slot = [&](int32_t *tg, int slot, int G, int seen) {
                if (seen != G + 1) {
                    ++waited;
                    const uint64_t t0 = wall_clock64();
                    uint32_t n = 0;
                    while (__hip_atomic_load(&tg[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != G + 1) {
                        if (spin_guard(a.flags, t0, n, a.wait_limit)) break;
                        __builtin_amdgcn_s_sleep(0);
                    }
                }
                // LDS only: the slot's data were written before the tag (see the loader)
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
            };
            auto load_ops = [&](T *nf, int slot) {
                const T *sl = ring + (size_t)slot * slot_elems;
#pragma unroll
                for (int e = 0; e < NE; ++e) nf[e] = sl[e * 64 + L];
            };
            int slot = gstep % D;                                   // slot of the current step
            // Step t with operands f (already in registers).  Order: neighbour
            // reads and the next slot's tag; the cell update; result writes;
            // release of this step's slot (its reads are consumed and its
            // results written); the next step's operands into fn (they land
            // while the face stores below are issued).
            int fseen = 0;   // face tag of the current step's slot, read one step ahead
            auto step = [&](const T *f, T *fn, int t) {
                const int G = gstep + t;
                const int nslot = slot + 1 == D ? 0 : slot + 1;
                const int pslot = slot == 0 ? D - 1 : slot - 1;   // the previous step's slot
                wait_slot(ftags, slot, G, fseen);   // the boundary lanes read this step's faces
                const T *bx = (const T *)(smem + (cx ? (uint32_t)slot * slot_bytes + xo_face : (uint32_t)pslot * slot_bytes + xo_int));
                const T *by = (const T *)(smem + (cy ? (uint32_t)slot * slot_bytes + yo_face : (uint32_t)pslot * slot_bytes + yo_int));
                T vx[3], vy[3];
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    vx[p] = bx[p];
                    vy[p] = by[p];
                }
                const bool more = t + 1 < nsteps;
                const int seen = more ? __hip_atomic_load(&tags[nslot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0;
                const int kk = DIR == 0 ? t - d : t - e_;
                const bool act = kk >= 0 && kk < nz;
                T out[3];
                if (DIR == 0) fwd_cell(f, last, vy, vx, f + 27, out);
                else bwd_cell(f, f + 27, vx, vy, last, f + 36, out);
                T *res = ring + (size_t)slot * slot_elems + RES;
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    out[p] = act ? out[p] : (T)0;
                    res[L * 3 + p] = out[p];
                    last[p] = out[p];
                }
                // this step's outgoing face words, from the result rows just written
                // (one wave: its LDS accesses complete in program order)
                const uint32_t fxv = half_bits(res[fx_src], fh);
                const uint32_t fyv = half_bits(res[fy_src], fh);
                // every read of this step's slot has been consumed and its results
                // written (the loader that refills the slot stores them): hand it back
                __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                if (L == 0) __hip_atomic_store(consumed, G + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                if (more) {
                    wait_slot(tags, nslot, G + 1, seen);
                    load_ops(fn, nslot);
                    fseen = __hip_atomic_load(&ftags[nslot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                // this step's face rows (row t - 7): the neighbouring tiles wait for them
                if ((unsigned)(t - fk0) < (unsigned)nz) {
                    const uint64_t ep = (uint64_t)a.epoch << 32;
                    if (fxw) face_st(fxo + (int64_t)(t - 7) * RW, ep | fxv);
                    if (fyw) face_st(fyo + (int64_t)(t - 7) * RW, ep | fyv);
                }
                slot = nslot;
            };
            T fa[NE], fb[NE];
            wait_slot(tags, slot, gstep, __hip_atomic_load(&tags[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            load_ops(fa, slot);
            fseen = __hip_atomic_load(&ftags[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            for (int t = 0; t < nsteps; t += 2) {
                if (a.trace && L == 0 && t == 8) a.trace[4 * T_ + 1] = wall_clock64();
                step(fa, fb, t);
                if (t + 1 >= nsteps) break;
                step(fb, fa, t + 1);
            }
            if (a.trace && L == 0) {
                a.trace[4 * T_ + 2] = wall_clock64();
                a.trace[4 * T_ + 3] = waited;
            }
        }
        gstep += nsteps;
        prevT = T_;
    }
    // loaders: the results of the last D steps are still in the ring
    if (wave > 0 && !aborted && prevT >= 0) {
        const int G0 = gstep - nsteps;   // first step of the last tile
        for (int G = gstep - D > G0 ? gstep - D : G0; G < gstep; ++G) {
            if (G % NLOAD != wave - 1) continue;
            if (__hip_atomic_load(consumed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < G + 1) {
                const uint64_t t0 = wall_clock64();
                uint32_t n = 0;
                while (__hip_atomic_load(consumed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < G + 1) {
                    if (spin_guard(a.flags, t0, n, a.wait_limit)) break;
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            store_results(ring + (size_t)(G % D) * slot_elems, prevT, G - G0);
        }
    }
}

// loader waves: 7, except the FP64 backward sweep whose 39-entry double
// buffers need the 512-register budget of a 4-wave workgroup
template <int DIR, typename T> struct NLoad { static constexpr int v = (DIR == 1 && sizeof(T) == 8) ? 3 : 7; };

template <typename T>
inline size_t sweep_slot_bytes(int dir)
{
    const int NS = (dir == 0) ? 30 : 40;   // entries per lane (+ the bwd output map entry)
    return (size_t)(NS * 64 + 48 + 192) * sizeof(T);   // + faces + the step's results
}
// dynamic LDS of a sweep: D ring slots and 64 tag words
template <typename T>
inline size_t sweep_lds_bytes(int dir, int D)
{
    return (size_t)D * sweep_slot_bytes<T>(dir) + 64 * sizeof(int32_t);
}

// zero n 64-bit words
__global__ __launch_bounds__(256) void k_zero_words(int64_t n, uint64_t *__restrict__ p)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0ull;
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
    int64_t face_words = 0;                      // words per face buffer
    int32_t *tile_order = nullptr;
    int64_t nbytes = 0;
    int btx = 0, bty = 0;                        // tiles per box (0: the whole grid)
    const int32_t *zmap = nullptr;               // optional output map of the pipelined apply (not owned)

    ~Bilu0() override
    {
        dev_free(Lf); dev_free(Dinv); dev_free(Lf32); dev_free(Dinv32); dev_free(U32);
        dev_free(ybuf); dev_free(zt32); dev_free(zt64); dev_free(faceX); dev_free(faceY); dev_free(tile_order);
        dev_free(trace);
    }
    int64_t bytes() const override { return nbytes; }

    rsv_status bilu0_factors(double *L, double *D) override
    {
        if (fp32 || !Lf || !Dinv) return set_err(c, RSV_ERR_ARG, "factors are kept for the FP64 BILU0 form only");
        const Geo &g = M->g->geo;
        const int64_t nc = M->g->ncell;
        double *buf = nullptr;
        rsv_status s = dev_alloc(c, (void **)&buf, (size_t)nc * 36 * sizeof(double));
        if (s != RSV_OK) return s;
        hipLaunchKernelGGL(k_factors_to_rows, dim3((unsigned)((g.nslot + BS - 1) / BS)), dim3(BS), 0, c->stream, g, Lf,
                           Dinv, buf, buf + nc * 27);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(L, buf, (size_t)nc * 27 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(D, buf + nc * 27, (size_t)nc * 9 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        dev_free(buf);
        if (e != hipSuccess) return set_err(c, RSV_ERR_HIP, std::string("factor export: ") + hipGetErrorString(e));
        return RSV_OK;
    }

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
        if (btx <= 0) btx = g.ntx;
        if (bty <= 0) bty = g.nty;
        if (g.ntx % btx != 0 || g.nty % bty != 0) return set_err(c, RSV_ERR_ARG, "boxes must tile the grid");
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
            face_words = (int64_t)NT * (g.nz + 7) * 24 * W;
            const size_t fb = (size_t)face_words * sizeof(uint64_t);
            // the sweeps keep a multi-slot ring in LDS: allow the full LDS per workgroup
            RSV_HIP(c, hipFuncSetAttribute((const void *)k_sweep<0, double, NLoad<0, double>::v>, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max));
            RSV_HIP(c, hipFuncSetAttribute((const void *)k_sweep<1, double, NLoad<1, double>::v>, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max));
            RSV_HIP(c, hipFuncSetAttribute((const void *)k_sweep<0, float, NLoad<0, float>::v>, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max));
            RSV_HIP(c, hipFuncSetAttribute((const void *)k_sweep<1, float, NLoad<1, float>::v>, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max));
            s = alloc((void **)&faceX, fb);
            if (s == RSV_OK) s = alloc((void **)&faceY, fb);
            if (s == RSV_OK) s = alloc((void **)&tile_order, (size_t)NT * sizeof(int32_t));
            if (s != RSV_OK) return s;
            // no word may carry a tag before its first write (epochs are never 0)
            const int nzb = (int)std::min<int64_t>((face_words + 255) / 256, 4096);
            hipLaunchKernelGGL(k_zero_words, dim3(nzb), dim3(256), 0, c->stream, face_words, faceX);
            hipLaunchKernelGGL(k_zero_words, dim3(nzb), dim3(256), 0, c->stream, face_words, faceY);
            RSV_LAUNCH(c);
            std::vector<int32_t> ord(NT);
            for (int t = 0; t < NT; ++t) ord[t] = t;
            // topological order: by anti-diagonal of the tile inside its box
            std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
                const int da = (a % g.ntx) % btx + (a / g.ntx) % bty, db = (b % g.ntx) % btx + (b / g.ntx) % bty;
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

    uint64_t *trace = nullptr;   // RSV_SWEEP_TRACE=<file>: per-tile timestamps of every pipelined sweep

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
        a.wait_limit = c->wait_ticks;
        a.btx = btx;
        a.bty = bty;
        a.trace = trace;
        c->ticket_base[0] += (uint64_t)(g.ntx * g.nty) + nwaves;
        return a;
    }

    // workgroups of the pipelined sweeps: one per CU (each holds a large LDS ring)
    int nwaves() const
    {
        const int NT = M->g->geo.ntx * M->g->geo.nty;
        return std::max(1, std::min(NT, c->num_cu));
    }

    void dump_trace(int dir)
    {
        const char *path = getenv("RSV_SWEEP_TRACE");
        if (!path || !trace) return;
        const int NT = M->g->geo.ntx * M->g->geo.nty;
        std::vector<uint64_t> h((size_t)NT * 4);
        if (hipStreamSynchronize(c->stream) != hipSuccess) return;
        if (hipMemcpy(h.data(), trace, h.size() * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess) return;
        FILE *fp = fopen(path, "a");
        if (!fp) return;
        fprintf(fp, "sweep dir=%d ntx=%d nty=%d nz=%d\n", dir, M->g->geo.ntx, M->g->geo.nty, M->g->geo.nz);
        for (int t = 0; t < NT; ++t)
            fprintf(fp, "%d %llu %llu %llu %llu\n", t, (unsigned long long)h[4 * t], (unsigned long long)h[4 * t + 1],
                    (unsigned long long)h[4 * t + 2], (unsigned long long)h[4 * t + 3]);
        fclose(fp);
    }

    rsv_status apply(const double *r, double *z) override
    {
        if (pipelined && getenv("RSV_SWEEP_TRACE") && !trace) {
            const int NT = M->g->geo.ntx * M->g->geo.nty;
            rsv_status s = alloc((void **)&trace, (size_t)NT * 4 * sizeof(uint64_t));
            if (s != RSV_OK) return s;
        }
        if (!pipelined) {
            ProfScope ps(c, RSV_K_ILU_FWD);
            if (fp32) return apply_plane<float>(r, z, Lf32, Dinv32, U32, zt32);
            return apply_plane<double>(r, z, Lf, Dinv, nullptr, zt64);
        }
        const Geo &g = M->g->geo;
        const int nw = nwaves();
        if (fp32) {
            SweepArgs a = sweep_args(nw);
            a.D = (int)sweep_ring_depth(c, 0, 1);
            SweepSrc<float> s0{Lf32, (int64_t)27 * 64, 0, nullptr, 0, 0, r, nullptr, nullptr};
            size_t sh = sweep_lds_bytes<float>(0, a.D);
            int t1 = prof_begin(c, RSV_K_ILU_FWD);
            hipLaunchKernelGGL((k_sweep<0, float, NLoad<0, float>::v>), dim3(nw), dim3(64 * (1 + NLoad<0, float>::v)), sh, c->stream, a, s0,
                               (float *)ybuf, (double *)nullptr);
            prof_end(c, t1);
            RSV_LAUNCH(c);
            SweepArgs b = sweep_args(nw);
            b.D = (int)sweep_ring_depth(c, 1, 1);
            SweepSrc<float> s1{U32, (int64_t)27 * 64, 0, Dinv32, (int64_t)9 * 64, 0, nullptr, (const float *)ybuf, zmap};
            sh = sweep_lds_bytes<float>(1, b.D);
            int t2 = prof_begin(c, RSV_K_ILU_BWD);
            hipLaunchKernelGGL((k_sweep<1, float, NLoad<1, float>::v>), dim3(nw), dim3(64 * (1 + NLoad<1, float>::v)), sh, c->stream, b, s1,
                               (float *)nullptr, z);
            prof_end(c, t2);
            RSV_LAUNCH(c);
        } else {
            SweepArgs a = sweep_args(nw);
            a.D = (int)sweep_ring_depth(c, 0, 0);
            SweepSrc<double> s0{Lf, (int64_t)27 * 64, 0, nullptr, 0, 0, r, nullptr, nullptr};
            size_t sh = sweep_lds_bytes<double>(0, a.D);
            int t1 = prof_begin(c, RSV_K_ILU_FWD);
            hipLaunchKernelGGL((k_sweep<0, double, NLoad<0, double>::v>), dim3(nw), dim3(64 * (1 + NLoad<0, double>::v)), sh, c->stream, a, s0,
                               (double *)ybuf, (double *)nullptr);
            prof_end(c, t1);
            RSV_LAUNCH(c);
            dump_trace(0);
            SweepArgs b = sweep_args(nw);
            b.D = (int)sweep_ring_depth(c, 1, 0);
            SweepSrc<double> s1{M->d_A, (int64_t)63 * 64, (int64_t)36 * 64, Dinv, (int64_t)9 * 64, 0, nullptr,
                                (const double *)ybuf, zmap};
            sh = sweep_lds_bytes<double>(1, b.D);
            int t2 = prof_begin(c, RSV_K_ILU_BWD);
            hipLaunchKernelGGL((k_sweep<1, double, NLoad<1, double>::v>), dim3(nw), dim3(64 * (1 + NLoad<1, double>::v)), sh, c->stream, b, s1,
                               (double *)nullptr, z);
            prof_end(c, t2);
            RSV_LAUNCH(c);
            dump_trace(1);
        }
        (void)g;
        return RSV_OK;
    }
};

}  // namespace

int64_t sweep_ring_depth(const rsv_ctx *c, int dir, int fp32)
{
    const size_t cap = (size_t)c->lds_max - 64 * sizeof(int32_t);
    const size_t sb = fp32 ? sweep_slot_bytes<float>(dir) : sweep_slot_bytes<double>(dir);
    return (int64_t)std::max<size_t>(2, std::min<size_t>(12, cap / sb));
}

rsv_status bilu0_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell)
{
    return bilu0_create_boxed(A, p, 0, 0, nullptr, out, bad_cell);
}

rsv_status bilu0_create_boxed(rsv_matrix *A, const rsv_pc_params *p, int btx, int bty, const int32_t *zmap,
                              PcImpl **out, int64_t *bad_cell)
{
    rsv_ctx *c = A->g->ctx;
    Bilu0 *B = new (std::nothrow) Bilu0();
    if (!B) return set_err(c, RSV_ERR_OOM, "bilu0");
    B->M = A;
    B->c = c;
    B->fp32 = (p->precision == RSV_FP32);
    B->pipelined = (p->pipelined != 0);
    B->btx = btx;
    B->bty = bty;
    B->zmap = zmap;
    if (zmap && !B->pipelined) {
        delete B;
        return set_err(c, RSV_ERR_ARG, "an output map needs the pipelined sweeps");
    }
    rsv_status s = B->setup(bad_cell);
    if (s != RSV_OK) {
        delete B;
        return s;
    }
    *out = B;
    return RSV_OK;
}
