// Bandwidth-bound kernels on the tile-lane layout: block SpMV with fused
// epilogues, layout permutes, assembly, and the vector operations of the
// Krylov drivers (Algebraic Operations: y = aAx + by, y = ax + by, <x,y>,
// ||x||) with deterministic two-stage reductions.
#include "rsv_internal.h"

#include <algorithm>

namespace {

constexpr int BS = 256;          // threads per block for streaming kernels
constexpr int RED_T = 1024;      // threads of the final reduction

// One stage of the halving reduction of H pairs of per-lane values: lanes
// whose bit `off` is set keep the upper half, the others the lower half, and
// each adds its partner's copy of the half it keeps; then the next stage.
template <int H>
__device__ __forceinline__ void halve(double *acc, int lane, int off)
{
    if constexpr (H >= 1) {
        const bool upper = (lane & off) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const double lo = acc[i], hi = acc[i + H];
            acc[i] = (upper ? hi : lo) + __shfl_xor(upper ? lo : hi, off, 64);
        }
        halve<H / 2>(acc, lane, off >> 1);
    }
}

constexpr int pow2_at_least(int k) { return k <= 1 ? 1 : 2 * pow2_at_least((k + 1) / 2); }
constexpr int log2_exact(int p) { return p <= 1 ? 0 : 1 + log2_exact(p / 2); }

// Wave part of a block sum of the first K of KB per-lane values (KB <= 64):
// value i summed over the wave's 64 lanes goes to red[(base + i) * nw + wave].
// The values (padded with zeros to P, a power of two) are halved over log2 P
// stages, so each shuffle moves a value that is still needed (P - 1 shuffles
// instead of 6 per value), and the remaining 64 / P lanes holding a value
// finish with plain butterflies.  Every value meets its partners in the same
// pairwise tree as a butterfly (a + b and b + a are the same double), so the
// sums equal the butterfly's bit for bit.
template <int KB>
__device__ inline void wave_sums_to(const double *acc_in, int K, double *red, int base)
{
    constexpr int P = pow2_at_least(KB);
    constexpr int S = log2_exact(P);
    constexpr int off = 32 >> S;   // butterfly distance left after the halving (0 when P = 64)
    static_assert(P <= 64, "at most 64 values per lane");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double acc[P];
#pragma unroll
    for (int i = 0; i < P; ++i) acc[i] = (i < KB) ? acc_in[i] : 0.0;
    halve<P / 2>(acc, lane, 32);
    double v = acc[0];
#pragma unroll
    for (int o = off; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    int idx = 0;   // the value this lane now holds
#pragma unroll
    for (int st = 0; st < S; ++st)
        if (lane & (32 >> st)) idx += (P / 2) >> st;
    if ((lane & (off ? 2 * off - 1 : 0)) == 0 && idx < K) red[(base + idx) * nw + w] = v;
}

// Block part, after a barrier: thread i < nout adds the waves' sums in wave order.
__device__ inline void block_finish(int nout, const double *red, double *out)
{
    const int nw = blockDim.x >> 6;
    if ((int)threadIdx.x < nout) {
        double t = 0.0;
        for (int q = 0; q < nw; ++q) t += red[threadIdx.x * nw + q];
        out[threadIdx.x] = t;
    }
}

// Sums of K per-thread values over the block, one barrier for all K (red holds
// KB * waves doubles).  Writes out[i], i < K.
template <int KB>
__device__ inline void block_sums(const double *acc, int K, double *red, double *out)
{
    wave_sums_to<KB>(acc, K, red, 0);
    __syncthreads();
    block_finish(K, red, out);
}

// Sum of v over the block (deterministic butterfly + fixed-order LDS pass);
// result valid in thread 0.
__device__ inline double block_sum(double v, double *lds)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < nw; ++q) s += lds[q];
    return s;
}

template <int MODE>
__global__ __launch_bounds__(BS) void k_spmv(Geo g, const double *__restrict__ A, const double *__restrict__ x,
                                             double *__restrict__ y, const double *__restrict__ aux1,
                                             double alpha, double beta, double *__restrict__ partials)
{
    __shared__ double lds[16];
    const int64_t slot = (int64_t)blockIdx.x * BS + threadIdx.x;
    const bool valid = slot < g.nslot;
    int gx = 0, gy = 0, k = 0;
    const bool real = valid && cell_of(g, slot, gx, gy, k);
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
                x0 = x[vidx(ns, 0)];
                x1 = x[vidx(ns, 1)];
                x2 = x[vidx(ns, 2)];
            }
            const double *a = A + aidx(slot, s * 9);
            acc0 += a[0 * 64] * x0 + a[1 * 64] * x1 + a[2 * 64] * x2;
            acc1 += a[3 * 64] * x0 + a[4 * 64] * x1 + a[5 * 64] * x2;
            acc2 += a[6 * 64] * x0 + a[7 * 64] * x1 + a[8 * 64] * x2;
        }
    }
    double r0 = 0.0, r1 = 0.0;
    if (valid) {
        double o0 = acc0, o1 = acc1, o2 = acc2;
        const int64_t i0 = vidx(slot, 0), i1 = vidx(slot, 1), i2 = vidx(slot, 2);
        if (MODE == SPMV_AXPBY) {
            o0 *= alpha; o1 *= alpha; o2 *= alpha;
            if (beta != 0.0) { o0 += beta * y[i0]; o1 += beta * y[i1]; o2 += beta * y[i2]; }
        } else if (MODE == SPMV_RESID) {
            o0 = aux1[i0] - acc0; o1 = aux1[i1] - acc1; o2 = aux1[i2] - acc2;
        }
        y[i0] = o0; y[i1] = o1; y[i2] = o2;
        if (MODE == SPMV_RESID || MODE == SPMV_NORM) r0 = o0 * o0 + o1 * o1 + o2 * o2;
        if (MODE == SPMV_DOT1 || MODE == SPMV_DOT2) r0 = aux1[i0] * o0 + aux1[i1] * o1 + aux1[i2] * o2;
        if (MODE == SPMV_DOT2) r1 = o0 * o0 + o1 * o1 + o2 * o2;
    }
    if (MODE >= SPMV_RESID) {
        const int K = (MODE == SPMV_DOT2) ? 2 : 1;
        double s0 = block_sum(r0, lds);
        if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * K] = s0;
        if (MODE == SPMV_DOT2) {
            double s1 = block_sum(r1, lds);
            if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * K + 1] = s1;
        }
    }
}

// final stage over the nb block partials ([nb][K]), fixed order: one
// workgroup per output, thread t sums partials t, t + RED_T, ... (loads
// issued eight at a time), then the block sum.
__global__ __launch_bounds__(RED_T) void k_reduce(const double *__restrict__ partials, int nb, int K,
                                                 double *__restrict__ out)
{
    __shared__ double lds[RED_T / 64];
    const int kk = blockIdx.x;
    double s = 0.0;
#pragma unroll 8
    for (int b = threadIdx.x; b < nb; b += RED_T) s += partials[(int64_t)b * K + kk];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[kk] = s;
}

__global__ __launch_bounds__(BS) void k_nat_to_tl(Geo g, const double *__restrict__ nat, double *__restrict__ tl)
{
    const int64_t slot = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (slot >= g.nslot) return;
    int gx, gy, k;
    const bool real = cell_of(g, slot, gx, gy, k);
    const int64_t row = real ? row_of(g, gx, gy, k) : 0;
    for (int p = 0; p < 3; ++p) tl[vidx(slot, p)] = real ? nat[3 * row + p] : 0.0;
}

__global__ __launch_bounds__(BS) void k_tl_to_nat(Geo g, const double *__restrict__ tl, double *__restrict__ nat,
                                                  double alpha, double beta)
{
    const int64_t slot = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (slot >= g.nslot) return;
    int gx, gy, k;
    if (!cell_of(g, slot, gx, gy, k)) return;
    const int64_t row = row_of(g, gx, gy, k);
    for (int p = 0; p < 3; ++p) {
        double v = alpha * tl[vidx(slot, p)];
        if (beta != 0.0) v += beta * nat[3 * row + p];
        nat[3 * row + p] = v;
    }
}

__global__ __launch_bounds__(BS) void k_assemble(Geo g, const double *__restrict__ blocks, double *__restrict__ A,
                                                 int32_t *flags)
{
    const int64_t slot = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (slot >= g.nslot) return;
    int gx, gy, k;
    const bool real = cell_of(g, slot, gx, gy, k);
    const int64_t row = real ? row_of(g, gx, gy, k) : 0;
    int bad = 0;
    for (int s = 0; s < 7; ++s) {
        int di, dj, dk;
        dir_off(s, di, dj, dk);
        const bool exists = real && gx + di >= 0 && gx + di < g.nx && gy + dj >= 0 && gy + dj < g.ny &&
                            k + dk >= 0 && k + dk < g.nz;
        for (int e = 0; e < 9; ++e) {
            const double v = real ? blocks[row * 63 + s * 9 + e] : 0.0;
            if (!isfinite(v)) bad |= FLAG_NAN;
            if (real && !exists && v != 0.0) bad |= FLAG_PATTERN;
            A[aidx(slot, s * 9 + e)] = exists ? v : 0.0;
        }
    }
    if (bad) atomicOr(&flags[0], bad);
}

// ---------------------------------------------------------------- vector ops

__global__ __launch_bounds__(BS) void k_dot(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                                            double *__restrict__ partials)
{
    __shared__ double lds[16];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS) s += x[e] * y[e];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(BS) void k_nonfinite(int64_t n, const double *__restrict__ x, double *__restrict__ partials)
{
    __shared__ double lds[16];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS)
        s += isfinite(x[e]) ? 0.0 : 1.0;
    s = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(BS) void k_copy(int64_t n, const double *__restrict__ x, double *__restrict__ y)
{
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS) y[e] = x[e];
}

__global__ __launch_bounds__(BS) void k_scale_dev(int64_t n, double *__restrict__ x, const double *__restrict__ sc)
{
    const double nn = sc[0];
    const double f = (nn > 0.0) ? 1.0 / sqrt(nn) : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS) x[e] *= f;
}

__global__ __launch_bounds__(BS) void k_axpby(int64_t n, double a, const double *__restrict__ x, double b,
                                              double *__restrict__ y)
{
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS)
        y[e] = (b == 0.0) ? a * x[e] : a * x[e] + b * y[e];
}

constexpr int KMAX = 64;   // max vectors in a multi-dot (GMRES restart <= 60)

// The multi-vector kernels load all KB vectors of an element unconditionally,
// vector index clamped to K-1 (in bounds; the extra terms are multiplied by a
// zero coefficient or their sums are discarded), so the loads are issued back
// to back instead of one branch -- and one memory round trip -- per vector.
__device__ __forceinline__ int64_t vrow(int i, int K, int64_t ldv) { return (int64_t)(i < K ? i : K - 1) * ldv; }

// partial dots V_i . w for i < K
template <int KB>
__global__ __launch_bounds__(BS) void k_mdot(int64_t n, const double *__restrict__ V, int64_t ldv, int K,
                                             const double *__restrict__ w, double *__restrict__ partials)
{
    __shared__ double red[KB * (BS / 64)];
    double acc[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) acc[i] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS) {
        double v[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) v[i] = V[vrow(i, K, ldv) + e];
        const double we = w[e];
#pragma unroll
        for (int i = 0; i < KB; ++i) acc[i] += v[i] * we;
    }
    block_sums<KB>(acc, K, red, partials + (int64_t)blockIdx.x * K);
}

// The second and third classical Gram-Schmidt passes over the basis, with
// coefficient sets c1 (the first pass's dots) and c2 (the second's):
//   MODE 0: u = w - sum_i c1_i V_i (ascending i), formed in registers only,
//           and the partial dots V_i . u;
//   MODE 1: w <- (w - sum_i c1_i V_i) - sum_i c2_i V_i (each sum ascending)
//           and the partial w . w.
// The pair gives the same bits as w -= V c1; dots; w -= V c2; norm, but the
// second pass only reads: a pass that also writes a stream runs at about
// 5 TB/s on this part, one that only reads at about 6.2.
template <int KB, int MODE>
__global__ __launch_bounds__(BS) void k_upd(int64_t n, const double *__restrict__ V, int64_t ldv, int K,
                                            double *__restrict__ w, const double *__restrict__ c1,
                                            const double *__restrict__ c2, double *__restrict__ partials)
{
    __shared__ double red[(MODE == 0 ? KB : 1) * (BS / 64)];
    double coef[KB], coef2[MODE == 1 ? KB : 1];
    double acc[MODE == 0 ? KB : 1];
#pragma unroll
    for (int i = 0; i < KB; ++i) coef[i] = (i < K) ? c1[i] : 0.0;
#pragma unroll
    for (int i = 0; i < (MODE == 1 ? KB : 1); ++i) coef2[i] = (MODE == 1 && i < K) ? c2[i] : 0.0;
#pragma unroll
    for (int i = 0; i < (MODE == 0 ? KB : 1); ++i) acc[i] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS) {
        double v[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) v[i] = V[vrow(i, K, ldv) + e];
        double we = w[e];
#pragma unroll
        for (int i = 0; i < KB; ++i) we -= coef[i] * v[i];
        if (MODE == 0) {
#pragma unroll
            for (int i = 0; i < KB; ++i) acc[i] += v[i] * we;
        } else {
#pragma unroll
            for (int i = 0; i < KB; ++i) we -= coef2[i] * v[i];
            w[e] = we;
            acc[0] += we * we;
        }
    }
    const int nout = (MODE == 0) ? K : 1;
    block_sums<(MODE == 0 ? KB : 1)>(acc, nout, red, partials + (int64_t)blockIdx.x * nout);
}

template <int KB>
__global__ __launch_bounds__(BS) void k_combine(int64_t n, const double *__restrict__ V, int64_t ldv, int K,
                                                const double *__restrict__ y, double *__restrict__ u, int accumulate)
{
    double coef[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) coef[i] = (i < K) ? y[i] : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS) {
        double v[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) v[i] = V[vrow(i, K, ldv) + e];
        double s = accumulate ? u[e] : 0.0;
#pragma unroll
        for (int i = 0; i < KB; ++i) s += coef[i] * v[i];
        u[e] = s;
    }
}

// DCGS2, first pass of step j (K = j + 1): partial dots V_i . V_{K-1} and
// V_i . w for i < K in one read of the basis.  Block b writes its 2K sums
// at partials[b * 2K]: the K dots with V_{K-1}, then the K dots with w.
template <int KB>
__global__ __launch_bounds__(BS) void k_dcgs_dots(int64_t n, const double *__restrict__ V, int64_t ldv, int K,
                                                  const double *__restrict__ w, double *__restrict__ partials)
{
    __shared__ double red[2 * KB * (BS / 64)];
    double ap[KB], aw[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) ap[i] = aw[i] = 0.0;
    const double *p = V + (int64_t)(K - 1) * ldv;
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS) {
        double v[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) v[i] = V[vrow(i, K, ldv) + e];
        const double pe = p[e], we = w[e];
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            ap[i] += v[i] * pe;
            aw[i] += v[i] * we;
        }
    }
    wave_sums_to<KB>(ap, K, red, 0);
    wave_sums_to<KB>(aw, K, red, K);
    __syncthreads();
    block_finish(2 * K, red, partials + (int64_t)blockIdx.x * 2 * K);
}

// DCGS2, second pass of step j (K = j + 1).  From the reduced dots d (s_i =
// d[i], t_i = d[K + i]) and omega = ||w||^2, every thread forms the same step
// scalars: beta = sqrt(d[j] - s.s) (1 at j = 0), u_j = (d[K + j] - s.t) / beta,
// d2 = omega - t.t - u_j^2.  Then per element
//     V_j <- (V_j - sum_{i<j} s_i V_i) / beta            (the delayed second pass on V_j)
//     w   <- (w - sum_{i<j} t_i V_i - u_j V_j) / sqrt(d2) (the first pass on w, normalised)
// with w <- 0 when d2 <= 64 eps omega (the norm is lost to rounding: breakdown).
// Block 0 stores beta, u_j, d2, omega at d[2K ..].
template <int KB>
__global__ __launch_bounds__(BS) void k_dcgs_upd(int64_t n, double *__restrict__ V, int64_t ldv, int K,
                                                 double *__restrict__ w, double *__restrict__ sc, int kd)
{
    const double *d = sc + kd;
    const int j = K - 1;
    double cs[KB], ct[KB];
    double ss = 0.0, st = 0.0, tt = 0.0;
#pragma unroll
    for (int i = 0; i < KB; ++i) {
        cs[i] = (i < j) ? d[i] : 0.0;
        ct[i] = (i < j) ? d[K + i] : 0.0;
        ss += cs[i] * cs[i];
        st += cs[i] * ct[i];
        tt += ct[i] * ct[i];
    }
    const double omega = sc[SC_W0];
    const double a = d[j] - ss;
    const double beta = (j == 0 || !(a > 0.0)) ? 1.0 : sqrt(a);
    const double ib = 1.0 / beta;
    const double uj = (d[K + j] - st) * ib;
    const double d2 = omega - (tt + uj * uj);
    const double scale = (d2 > DCGS_LOST * omega) ? 1.0 / sqrt(d2) : 0.0;
    double *p = V + (int64_t)j * ldv;
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS) {
        double v[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) v[i] = V[vrow(i, K, ldv) + e];
        double q = p[e], we = w[e];
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            q -= cs[i] * v[i];
            we -= ct[i] * v[i];
        }
        q *= ib;
        if (j > 0) p[e] = q;
        w[e] = (we - uj * q) * scale;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[kd + 2 * K] = beta;
        sc[kd + 2 * K + 1] = uj;
        sc[kd + 2 * K + 2] = d2;
        sc[kd + 2 * K + 3] = omega;
    }
}

__global__ __launch_bounds__(BS) void k_bicg_p(int64_t n, const double *__restrict__ r, const double *__restrict__ v,
                                               double beta, double omega, double *__restrict__ p)
{
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS)
        p[e] = r[e] + beta * (p[e] - omega * v[e]);
}

__global__ __launch_bounds__(BS) void k_bicg_s(int64_t n, const double *__restrict__ r, const double *__restrict__ v,
                                               double *__restrict__ s, const double *__restrict__ sc, int knum,
                                               int kden, double *__restrict__ partials)
{
    __shared__ double lds[16];
    const double alpha = sc[knum] / sc[kden];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS) {
        const double se = r[e] - alpha * v[e];
        s[e] = se;
        acc += se * se;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// omega = sc[SC_TS] / sc[SC_TT] (0 when tt = 0); x += alpha ph + omega sh; r = s - omega t
__global__ __launch_bounds__(BS) void k_bicg_xr(int64_t n, double alpha, const double *__restrict__ sc,
                                                const double *__restrict__ ph, const double *__restrict__ sh,
                                                const double *__restrict__ s, const double *__restrict__ t,
                                                const double *__restrict__ rh, double *__restrict__ x,
                                                double *__restrict__ r, double *__restrict__ partials)
{
    __shared__ double lds[16];
    const double tt = sc[SC_TT];
    const double omega = (tt > 0.0) ? sc[SC_TS] / tt : 0.0;
    double a0 = 0.0, a1 = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS) {
        x[e] += alpha * ph[e] + omega * sh[e];
        const double re = s[e] - omega * t[e];
        r[e] = re;
        a0 += re * re;
        a1 += rh[e] * re;
    }
    a0 = block_sum(a0, lds);
    if (threadIdx.x == 0) partials[2 * blockIdx.x] = a0;
    a1 = block_sum(a1, lds);
    if (threadIdx.x == 0) partials[2 * blockIdx.x + 1] = a1;
}

}  // namespace

// ---------------------------------------------------------------- launchers

#ifndef RSV_MVEC_BLOCKS
#define RSV_MVEC_BLOCKS 4096
#endif

rsv_status partials_reserve(rsv_ctx *c, int64_t nd)
{
    if (nd <= c->partials_cap) return RSV_OK;
    // Growing needs a stream sync (the stream may still read the old buffer),
    // so grow rarely: at least 2 MiB (RSV_MVEC_BLOCKS blocks x 64 outputs) and
    // at least twice the old size.
    nd = std::max<int64_t>(nd, std::max<int64_t>((int64_t)RSV_MVEC_BLOCKS * 64, 2 * c->partials_cap));
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    if (c->d_partials) dev_free(c->d_partials);
    c->d_partials = nullptr;
    c->partials_cap = 0;
    rsv_status s = dev_alloc(c, (void **)&c->d_partials, (size_t)nd * sizeof(double));
    if (s != RSV_OK) return s;
    c->partials_cap = nd;
    return RSV_OK;
}

int spmv_blocks(const Geo &g) { return (int)((g.nslot + BS - 1) / BS); }
int vec_blocks(int64_t n)
{
    int64_t b = (n + BS - 1) / BS;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 2048);
}

// the multi-vector (CGS2) kernels (grid size chosen by measurement)
int mvec_blocks(int64_t n)
{
    int64_t b = (n + BS - 1) / BS;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), RSV_MVEC_BLOCKS);
}

rsv_status launch_reduce(rsv_ctx *c, int nblocks, int K, int k0)
{
    if (K <= 0) return RSV_OK;
    hipLaunchKernelGGL(k_reduce, dim3(K), dim3(RED_T), 0, c->stream, c->d_partials, nblocks, K, c->d_scal + k0);
    RSV_LAUNCH(c);
    return RSV_OK;
}

rsv_status launch_spmv(rsv_ctx *c, const Geo &g, const double *A, int mode, const double *x, double *y,
                       const double *aux1, double alpha, double beta, int k0)
{
    const int nb = spmv_blocks(g);
    if (mode >= SPMV_RESID) {
        rsv_status s = partials_reserve(c, (int64_t)nb * 2);
        if (s != RSV_OK) return s;
    }
    dim3 grid(nb), block(BS);
    double *P = c->d_partials;
    const int tok = prof_begin(c, RSV_K_SPMV);
    switch (mode) {
    case SPMV_Y: hipLaunchKernelGGL(k_spmv<SPMV_Y>, grid, block, 0, c->stream, g, A, x, y, aux1, alpha, beta, P); break;
    case SPMV_AXPBY: hipLaunchKernelGGL(k_spmv<SPMV_AXPBY>, grid, block, 0, c->stream, g, A, x, y, aux1, alpha, beta, P); break;
    case SPMV_RESID: hipLaunchKernelGGL(k_spmv<SPMV_RESID>, grid, block, 0, c->stream, g, A, x, y, aux1, alpha, beta, P); break;
    case SPMV_NORM: hipLaunchKernelGGL(k_spmv<SPMV_NORM>, grid, block, 0, c->stream, g, A, x, y, aux1, alpha, beta, P); break;
    case SPMV_DOT1: hipLaunchKernelGGL(k_spmv<SPMV_DOT1>, grid, block, 0, c->stream, g, A, x, y, aux1, alpha, beta, P); break;
    case SPMV_DOT2: hipLaunchKernelGGL(k_spmv<SPMV_DOT2>, grid, block, 0, c->stream, g, A, x, y, aux1, alpha, beta, P); break;
    default: return set_err(c, RSV_ERR_ARG, "bad spmv mode");
    }
    prof_end(c, tok);
    RSV_LAUNCH(c);
    if (mode >= SPMV_RESID) return launch_reduce(c, nb, mode == SPMV_DOT2 ? 2 : 1, k0);
    return RSV_OK;
}

rsv_status launch_nat_to_tl(rsv_ctx *c, const Geo &g, const double *nat, double *tl)
{
    hipLaunchKernelGGL(k_nat_to_tl, dim3(spmv_blocks(g)), dim3(BS), 0, c->stream, g, nat, tl);
    RSV_LAUNCH(c);
    return RSV_OK;
}

rsv_status launch_tl_to_nat(rsv_ctx *c, const Geo &g, const double *tl, double *nat, double alpha, double beta)
{
    hipLaunchKernelGGL(k_tl_to_nat, dim3(spmv_blocks(g)), dim3(BS), 0, c->stream, g, tl, nat, alpha, beta);
    RSV_LAUNCH(c);
    return RSV_OK;
}

rsv_status launch_assemble(rsv_ctx *c, const Geo &g, const double *blocks, double *A)
{
    hipLaunchKernelGGL(k_assemble, dim3(spmv_blocks(g)), dim3(BS), 0, c->stream, g, blocks, A, c->d_flags);
    RSV_LAUNCH(c);
    return RSV_OK;
}

rsv_status launch_dot(rsv_ctx *c, int64_t n, const double *x, const double *y, int k0)
{
    const int nb = vec_blocks(n);
    rsv_status s = partials_reserve(c, nb);
    if (s != RSV_OK) return s;
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(BS), 0, c->stream, n, x, y, c->d_partials);
    RSV_LAUNCH(c);
    return launch_reduce(c, nb, 1, k0);
}

rsv_status launch_nonfinite(rsv_ctx *c, int64_t n, const double *x, int k0)
{
    const int nb = vec_blocks(n);
    rsv_status s = partials_reserve(c, nb);
    if (s != RSV_OK) return s;
    hipLaunchKernelGGL(k_nonfinite, dim3(nb), dim3(BS), 0, c->stream, n, x, c->d_partials);
    RSV_LAUNCH(c);
    return launch_reduce(c, nb, 1, k0);
}

rsv_status launch_copy(rsv_ctx *c, int64_t n, const double *x, double *y)
{
    hipLaunchKernelGGL(k_copy, dim3(vec_blocks(n)), dim3(BS), 0, c->stream, n, x, y);
    RSV_LAUNCH(c);
    return RSV_OK;
}

rsv_status launch_scale_dev(rsv_ctx *c, int64_t n, double *x, int k)
{
    ProfScope ps(c, RSV_K_ORTHO);
    hipLaunchKernelGGL(k_scale_dev, dim3(vec_blocks(n)), dim3(BS), 0, c->stream, n, x, c->d_scal + k);
    RSV_LAUNCH(c);
    return RSV_OK;
}

rsv_status launch_axpby(rsv_ctx *c, int64_t n, double a, const double *x, double b, double *y)
{
    hipLaunchKernelGGL(k_axpby, dim3(vec_blocks(n)), dim3(BS), 0, c->stream, n, a, x, b, y);
    RSV_LAUNCH(c);
    return RSV_OK;
}

#define KB_DISPATCH(K, MACRO) \
    if ((K) <= 8) { MACRO(8); } else if ((K) <= 16) { MACRO(16); } else if ((K) <= 24) { MACRO(24); } \
    else if ((K) <= 32) { MACRO(32); } else if ((K) <= 40) { MACRO(40); } else if ((K) <= 48) { MACRO(48); } \
    else if ((K) <= 56) { MACRO(56); } else { MACRO(64); }

rsv_status launch_mdot(rsv_ctx *c, int64_t n, const double *V, int64_t ldv, int K, const double *w, int k0)
{
    if (K < 1 || K > KMAX) return set_err(c, RSV_ERR_ARG, "mdot K");
    const int nb = mvec_blocks(n);
    rsv_status s = partials_reserve(c, (int64_t)nb * K);
    if (s != RSV_OK) return s;
#define L_MDOT(KB) hipLaunchKernelGGL(k_mdot<KB>, dim3(nb), dim3(BS), 0, c->stream, n, V, ldv, K, w, c->d_partials)
    {
        ProfScope ps(c, RSV_K_ORTHO);
        KB_DISPATCH(K, L_MDOT)
    }
#undef L_MDOT
    RSV_LAUNCH(c);
    return launch_reduce(c, nb, K, k0);
}

rsv_status launch_upd_dot(rsv_ctx *c, int64_t n, const double *V, int64_t ldv, int K, double *w, int kc, int k0)
{
    if (K < 1 || K > KMAX) return set_err(c, RSV_ERR_ARG, "upd K");
    const int nb = mvec_blocks(n);
    rsv_status s = partials_reserve(c, (int64_t)nb * K);
    if (s != RSV_OK) return s;
#define L_UPD(KB)                                                                                          \
    hipLaunchKernelGGL((k_upd<KB, 0>), dim3(nb), dim3(BS), 0, c->stream, n, V, ldv, K, w, c->d_scal + kc, \
                       c->d_scal + kc, c->d_partials)
    {
        ProfScope ps(c, RSV_K_ORTHO);
        KB_DISPATCH(K, L_UPD)
    }
#undef L_UPD
    RSV_LAUNCH(c);
    return launch_reduce(c, nb, K, k0);
}

rsv_status launch_upd_norm(rsv_ctx *c, int64_t n, const double *V, int64_t ldv, int K, double *w, int kc1, int kc2,
                           int k0)
{
    if (K < 1 || K > KMAX) return set_err(c, RSV_ERR_ARG, "upd K");
    const int nb = mvec_blocks(n);
    rsv_status s = partials_reserve(c, nb);
    if (s != RSV_OK) return s;
#define L_UPDN(KB)                                                                                          \
    hipLaunchKernelGGL((k_upd<KB, 1>), dim3(nb), dim3(BS), 0, c->stream, n, V, ldv, K, w, c->d_scal + kc1, \
                       c->d_scal + kc2, c->d_partials)
    {
        ProfScope ps(c, RSV_K_ORTHO);
        KB_DISPATCH(K, L_UPDN)
    }
#undef L_UPDN
    RSV_LAUNCH(c);
    return launch_reduce(c, nb, 1, k0);
}

rsv_status launch_combine(rsv_ctx *c, int64_t n, const double *V, int64_t ldv, int K, int ky, double *u, int accumulate)
{
    if (K < 1 || K > KMAX) return set_err(c, RSV_ERR_ARG, "combine K");
    const int nb = vec_blocks(n);
#define L_CMB(KB) hipLaunchKernelGGL(k_combine<KB>, dim3(nb), dim3(BS), 0, c->stream, n, V, ldv, K, c->d_scal + ky, u, accumulate)
    {
        ProfScope ps(c, RSV_K_ORTHO);
        KB_DISPATCH(K, L_CMB)
    }
#undef L_CMB
    RSV_LAUNCH(c);
    return RSV_OK;
}

rsv_status launch_dcgs_dots(rsv_ctx *c, int64_t n, const double *V, int64_t ldv, int K, const double *w, int k0)
{
    if (K < 1 || K > KMAX || k0 + 2 * K + 4 > SC_COUNT) return set_err(c, RSV_ERR_ARG, "dcgs K");
    const int nb = mvec_blocks(n);
    rsv_status s = partials_reserve(c, (int64_t)nb * 2 * K);
    if (s != RSV_OK) return s;
#define L_DD(KB) hipLaunchKernelGGL(k_dcgs_dots<KB>, dim3(nb), dim3(BS), 0, c->stream, n, V, ldv, K, w, c->d_partials)
    {
        ProfScope ps(c, RSV_K_ORTHO);
        KB_DISPATCH(K, L_DD)
    }
#undef L_DD
    RSV_LAUNCH(c);
    return launch_reduce(c, nb, 2 * K, k0);
}

rsv_status launch_dcgs_update(rsv_ctx *c, int64_t n, double *V, int64_t ldv, int K, double *w, int kd)
{
    if (K < 1 || K > KMAX || kd + 2 * K + 4 > SC_COUNT) return set_err(c, RSV_ERR_ARG, "dcgs K");
    const int nb = mvec_blocks(n);
#define L_DU(KB) hipLaunchKernelGGL(k_dcgs_upd<KB>, dim3(nb), dim3(BS), 0, c->stream, n, V, ldv, K, w, c->d_scal, kd)
    {
        ProfScope ps(c, RSV_K_ORTHO);
        KB_DISPATCH(K, L_DU)
    }
#undef L_DU
    RSV_LAUNCH(c);
    return RSV_OK;
}

rsv_status launch_bicg_p(rsv_ctx *c, int64_t n, const double *r, const double *v, double beta, double omega, double *p)
{
    ProfScope ps(c, RSV_K_VEC);
    hipLaunchKernelGGL(k_bicg_p, dim3(vec_blocks(n)), dim3(BS), 0, c->stream, n, r, v, beta, omega, p);
    RSV_LAUNCH(c);
    return RSV_OK;
}

rsv_status launch_bicg_s(rsv_ctx *c, int64_t n, const double *r, const double *v, double *s, int knum, int kden, int k0)
{
    const int nb = vec_blocks(n);
    rsv_status st = partials_reserve(c, nb);
    if (st != RSV_OK) return st;
    ProfScope ps(c, RSV_K_VEC);
    hipLaunchKernelGGL(k_bicg_s, dim3(nb), dim3(BS), 0, c->stream, n, r, v, s, c->d_scal, knum, kden, c->d_partials);
    RSV_LAUNCH(c);
    return launch_reduce(c, nb, 1, k0);
}

rsv_status launch_bicg_xr(rsv_ctx *c, int64_t n, double alpha, double /*omega_unused*/, const double *ph, const double *sh,
                          const double *s, const double *t, const double *rh, double *x, double *r, int k0)
{
    const int nb = vec_blocks(n);
    rsv_status st = partials_reserve(c, (int64_t)nb * 2);
    if (st != RSV_OK) return st;
    ProfScope ps(c, RSV_K_VEC);
    hipLaunchKernelGGL(k_bicg_xr, dim3(nb), dim3(BS), 0, c->stream, n, alpha, c->d_scal, ph, sh, s, t, rh, x, r,
                       c->d_partials);
    RSV_LAUNCH(c);
    return launch_reduce(c, nb, 2, k0);
}

rsv_status scal_to_host(rsv_ctx *c, int k0, int n)
{
    RSV_HIP(c, hipMemcpyAsync(c->h_scal + k0, c->d_scal + k0, (size_t)n * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    return RSV_OK;
}

rsv_status scal_to_host_async(rsv_ctx *c, int buf, int k0, int n)
{
    if (!c->h_spec) {
        RSV_HIP(c, hipHostMalloc((void **)&c->h_spec, 2 * SC_COUNT * sizeof(double), hipHostMallocDefault));
        for (int b = 0; b < 2; ++b) RSV_HIP(c, hipEventCreateWithFlags(&c->spec_ev[b], hipEventDisableTiming));
    }
    double *dst = c->h_spec + (size_t)buf * SC_COUNT;
    RSV_HIP(c, hipMemcpyAsync(dst + k0, c->d_scal + k0, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    RSV_HIP(c, hipEventRecord(c->spec_ev[buf], c->stream));
    return RSV_OK;
}

rsv_status scal_wait(rsv_ctx *c, int buf)
{
    RSV_HIP(c, hipEventSynchronize(c->spec_ev[buf]));
    return RSV_OK;
}

rsv_status scal_set(rsv_ctx *c, int k0, const double *vals, int n)
{
    // staged through the pinned buffer so the copy is truly asynchronous
    for (int i = 0; i < n; ++i) c->h_scal[k0 + i] = vals[i];
    RSV_HIP(c, hipMemcpyAsync(c->d_scal + k0, c->h_scal + k0, (size_t)n * sizeof(double), hipMemcpyHostToDevice,
                              c->stream));
    // the pinned slots may be overwritten by the next scal_to_host; make the copy complete first
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    return RSV_OK;
}
