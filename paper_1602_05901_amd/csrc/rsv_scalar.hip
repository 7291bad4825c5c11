// Scalar (one unknown per cell) 7-point systems, for the paper's Poisson
// Equation example: GMRES(30) with restricted additive Schwarz, overlap one,
// ILU(0) on every subdomain (Restricted Additive Schwarz Method subsection,
// RAS default parameters; Poisson Equation example).
//
// Storage: the seven coefficients of every row as seven row-ordered arrays
// coef[s][row] (slots -z,-y,-x,D,+x,+y,+z by cell direction), vectors in row
// order; the product is one thread per row with the residual, norm and dot
// epilogues of the block product.
//
// RAS: px x py x pz boxes (the first n mod p boxes one cell longer), each
// extended to Omega_s = the cells within graph distance `overlap` of the box
// (L1 distance on the lattice: faces, no edges or corners for overlap 1).
// The local ILU(0) in ascending global order has no fill on the 7-point graph
// (two neighbours of a cell are never neighbours), so D_c = a_cc -
// sum_{k lower} a_ck a_kc / D_k.  One workgroup per subdomain walks planes of
// x-chunks (each depending only on the plane before) with a barrier between
// them, for the factorisation and for both sweeps of an apply; only the
// owner of a cell writes its result.
#include "rsv_internal.h"

#include <algorithm>
#include <cmath>
#include <new>
#include <thread>
#include <vector>

namespace {

constexpr int SB = 256;          // product / assembly threads per block
constexpr int RAS_T = 1024;      // threads of a subdomain's workgroup (factorisation)
constexpr int APPLY_T = 512;     // threads of a subdomain's workgroup (apply: 8 slots of values per thread)

// row -> cell (inverse of row_of)
__host__ __device__ inline void cell_of_row(const Geo &g, int64_t r, int &i, int &j, int &k)
{
    i = (int)(r % g.nx);
    j = (int)((r / g.nx) % g.ny);
    const int kk = (int)(r / ((int64_t)g.nx * g.ny));
    k = (g.ordering == RSV_TOP_DOWN) ? g.nz - 1 - kk : kk;
}

__device__ inline double sblock_sum(double v, double *lds)
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

__global__ __launch_bounds__(SB) void k_sassemble(Geo g, const double *__restrict__ src, double *__restrict__ coef,
                                                  int32_t *flags)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t r = (int64_t)blockIdx.x * SB + threadIdx.x;
    if (r >= n) return;
    int i, j, k;
    cell_of_row(g, r, i, j, k);
    for (int s = 0; s < 7; ++s) {
        int di, dj, dk;
        dir_off(s, di, dj, dk);
        const bool inside = i + di >= 0 && i + di < g.nx && j + dj >= 0 && j + dj < g.ny && k + dk >= 0 && k + dk < g.nz;
        const double v = src[7 * r + s];
        if (!isfinite(v)) {
            atomicOr(&flags[0], (int32_t)FLAG_NAN);
            atomicMin(&flags[1], (int32_t)r);
        } else if (!inside && v != 0.0) {
            atomicOr(&flags[0], (int32_t)FLAG_PATTERN);
            atomicMin(&flags[1], (int32_t)r);
        }
        coef[s * n + r] = inside ? v : 0.0;
    }
}

template <int MODE>
__global__ __launch_bounds__(SB) void k_sspmv(Geo g, const double *__restrict__ coef, const double *__restrict__ x,
                                              double *__restrict__ y, const double *__restrict__ aux,
                                              double alpha, double beta, double *__restrict__ partials)
{
    __shared__ double lds[SB / 64];
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t r = (int64_t)blockIdx.x * SB + threadIdx.x;
    double r0 = 0.0, r1 = 0.0;
    if (r < n) {
        int i, j, k;
        cell_of_row(g, r, i, j, k);
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < 7; ++s) {
            int di, dj, dk;
            dir_off(s, di, dj, dk);
            const int a = i + di, b = j + dj, c = k + dk;
            if (a >= 0 && a < g.nx && b >= 0 && b < g.ny && c >= 0 && c < g.nz)
                acc += coef[s * n + r] * x[(s == 3) ? r : row_of(g, a, b, c)];
        }
        double o = acc;
        if (MODE == SPMV_AXPBY) {
            o *= alpha;
            if (beta != 0.0) o += beta * y[r];
        } else if (MODE == SPMV_RESID) {
            o = aux[r] - acc;
        }
        y[r] = o;
        if (MODE == SPMV_RESID || MODE == SPMV_NORM) r0 = o * o;
        if (MODE == SPMV_DOT1 || MODE == SPMV_DOT2) r0 = aux[r] * o;
        if (MODE == SPMV_DOT2) r1 = o * o;
    }
    if (MODE >= SPMV_RESID) {
        const int K = (MODE == SPMV_DOT2) ? 2 : 1;
        const double s0 = sblock_sum(r0, lds);
        if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * K] = s0;
        if (MODE == SPMV_DOT2) {
            const double s1 = sblock_sum(r1, lds);
            if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * K + 1] = s1;
        }
    }
}

// ---------------------------------------------------------------- RAS
// A subdomain is walked in chunks of SW consecutive x-cells: chunk (c, j, k)
// of the extended box [ex0, ex1) x [ey0, ey1) x [ez0, ez1) holds the cells
// x = ex0 + SW c + t (t < SW) of grid row (ey0 + j, ez0 + k).  The lower
// neighbours of its cells (x - 1 of slot 0, y - 1, z - 1) lie in chunks
// (c-1, j, k), (c, j-1, k) and (c, j, k-1), so chunk plane P = c + j + k
// depends only on plane P - 1, and one thread solves the slots of a chunk in
// x order: a topological order of the same triangular dependencies as the
// cell hyperplanes, with the same arithmetic per cell.  Only chunks holding
// an Omega_s cell are stored; a slot outside Omega_s (x beyond the extended
// box, or an edge or corner of it) has zero couplings, a zero pivot inverse
// and the value zero.
//
// Chunk arrays (grouped by subdomain, then by plane, inside a plane by
// (k, j, c)): row0 = row of slot 0; mask = bit t: slot t in Omega_s, bit
// OWN_SHIFT + t: slot t owned by the subdomain; nlo[q] = position inside
// plane P - 1 of the (c, j, k-1), (c, j-1, k), (c-1, j, k) chunk and nhi[q] =
// position inside plane P + 1 of the (c+1, j, k), (c, j+1, k), (c, j, k+1)
// chunk, or -1.  Slot arrays: l[q] = a_ck / D_k (q = -z, -y, -x), u[q] = a_cm
// (q = +x, +y, +z), dinv = 1 / D_c, y = the sweeps' values; slot t of the
// chunk at position p of plane P is element SW pl[P] + t n_P + p (n_P chunks
// in the plane), so one slot of a plane's chunks is one contiguous row.
constexpr int SW = 8;
constexpr int OWN_SHIFT = 16;

struct SRasDev {
    int64_t nitem;                     // chunks over all subdomains
    const int32_t *row0, *mask, *nlo, *nhi;
    double *l, *u, *dinv, *y;          // SW * nitem elements each (l and u: three arrays)
    const int64_t *pl;                 // pl[pl_off[s] + P]: first chunk of plane P of subdomain s
    const int32_t *pl_off, *pl_cnt;
};

__device__ constexpr int LO_SLOT[3] = {0, 1, 2};   // -z, -y, -x
__device__ constexpr int HI_SLOT[3] = {4, 5, 6};   // +x, +y, +z

// D_c = a_cc - sum over lower neighbours k in Omega_s of (a_ck / D_k) a_kc,
// plane by plane (the planes before P are final when P starts)
__global__ __launch_bounds__(RAS_T) void k_sras_factor(Geo g, const double *__restrict__ coef, SRasDev d,
                                                       int32_t *flags)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz, ns = SW * d.nitem;
    const int s = blockIdx.x, np = d.pl_cnt[s];
    const int64_t *pl = d.pl + d.pl_off[s];
    for (int P = 0; P < np; ++P) {
        const int64_t f = pl[P], cnt = pl[P + 1] - f;
        const int64_t fm = P > 0 ? pl[P - 1] : f, cm = f - fm;                  // plane P - 1
        const int64_t fp = pl[P + 1];                                          // plane P + 1
        for (int64_t p = threadIdx.x; p < cnt; p += RAS_T) {
            const int64_t q = f + p;
            const int64_t r0 = d.row0[q];
            const int m = d.mask[q];
            int32_t lo[3], hi[3];
            int lm[3], hm[3];
            int64_t lr[2];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = d.nlo[a * d.nitem + q];
                hi[a] = d.nhi[a * d.nitem + q];
                lm[a] = lo[a] >= 0 ? d.mask[fm + lo[a]] : 0;
                hm[a] = hi[a] >= 0 ? d.mask[fp + hi[a]] : 0;
            }
            lr[0] = lo[0] >= 0 ? d.row0[fm + lo[0]] : 0;
            lr[1] = lo[1] >= 0 ? d.row0[fm + lo[1]] : 0;
            // x - 1 of slot 0: slot SW - 1 of chunk lo[2]
            bool xl = lo[2] >= 0 && ((lm[2] >> (SW - 1)) & 1);
            double dxl = xl ? d.dinv[SW * fm + (SW - 1) * cm + lo[2]] : 0.0;
            for (int t = 0; t < SW; ++t) {
                const int64_t e = SW * f + t * cnt + p;
                if (!((m >> t) & 1)) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        d.l[a * ns + e] = 0.0;
                        d.u[a * ns + e] = 0.0;
                    }
                    d.dinv[e] = 0.0;
                    xl = false;
                    continue;
                }
                const int64_t r = r0 + t;
                double dd = coef[3 * n + r];
#pragma unroll
                for (int a = 0; a < 2; ++a) {            // -z, -y: slot t of chunks lo[0], lo[1]
                    double lv = 0.0;
                    if (lo[a] >= 0 && ((lm[a] >> t) & 1)) {
                        const double a_ck = coef[LO_SLOT[a] * n + r];
                        const double a_kc = coef[(6 - LO_SLOT[a]) * n + lr[a] + t];
                        lv = a_ck * d.dinv[SW * fm + t * cm + lo[a]];
                        dd -= lv * a_kc;
                    }
                    d.l[a * ns + e] = lv;
                }
                {                                        // -x: slot t - 1, or chunk lo[2]
                    double lv = 0.0;
                    if (xl) {
                        lv = coef[LO_SLOT[2] * n + r] * dxl;
                        dd -= lv * coef[(6 - LO_SLOT[2]) * n + r - 1];
                    }
                    d.l[2 * ns + e] = lv;
                }
                const bool up[3] = {t < SW - 1 ? (((m >> (t + 1)) & 1) != 0) : (hi[0] >= 0 && (hm[0] & 1)),
                                    hi[1] >= 0 && ((hm[1] >> t) & 1), hi[2] >= 0 && ((hm[2] >> t) & 1)};
#pragma unroll
                for (int a = 0; a < 3; ++a) d.u[a * ns + e] = up[a] ? coef[HI_SLOT[a] * n + r] : 0.0;
                double di;
                if (!(fabs(dd) > 1e-300) || !isfinite(dd)) {
                    atomicOr(&flags[0], (int32_t)FLAG_PIVOT);
                    atomicMin(&flags[1], (int32_t)r);
                    di = 0.0;
                } else {
                    di = 1.0 / dd;
                }
                d.dinv[e] = di;
                dxl = di;
                xl = true;
            }
        }
        __syncthreads();
    }
}

// ids of the chunk at position p of a plane (first chunk f, cnt chunks): row
// of slot 0, mask and three neighbour positions from nb; a position past the
// plane gets mask 0 and no neighbours
struct ChunkIds {
    int32_t r0, m, a, b, c;
};

__device__ inline ChunkIds chunk_ids(const SRasDev &d, const int32_t *nb, int64_t f, int64_t cnt, int64_t p)
{
    ChunkIds k{0, 0, -1, -1, -1};
    if (p < cnt) {
        const int64_t q = f + p;
        k.r0 = d.row0[q];
        k.m = d.mask[q];
        k.a = nb[q];
        k.b = nb[d.nitem + q];
        k.c = nb[2 * d.nitem + q];
    }
    return k;
}

// operands of one chunk's forward step: r, the z-1 and y-1 neighbours' values
// (plane P - 1: first chunk fm, cm chunks), the x-1 value of slot 0, l
struct FwdOps {
    double rv[SW], yz[SW], yy[SW], l[3][SW], yx;
};

__device__ inline void fwd_load(const SRasDev &d, const double *rin, const ChunkIds &k, int64_t f, int64_t cnt,
                                int64_t p, int64_t fm, int64_t cm, FwdOps &o)
{
    const int64_t ns = SW * d.nitem;
    const bool live = p < cnt;
#pragma unroll
    for (int t = 0; t < SW; ++t) {
        const int64_t e = SW * f + t * cnt + p;
        o.rv[t] = ((k.m >> t) & 1) ? rin[k.r0 + t] : 0.0;
        o.yz[t] = k.a >= 0 ? d.y[SW * fm + t * cm + k.a] : 0.0;
        o.yy[t] = k.b >= 0 ? d.y[SW * fm + t * cm + k.b] : 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) o.l[a][t] = live ? __builtin_nontemporal_load(d.l + a * ns + e) : 0.0;
    }
    o.yx = k.c >= 0 ? d.y[SW * fm + (SW - 1) * cm + k.c] : 0.0;
}

__device__ inline void fwd_solve(const SRasDev &d, int64_t f, int64_t cnt, int64_t p, const FwdOps &o)
{
    if (p >= cnt) return;
    double v = o.yx;
#pragma unroll
    for (int t = 0; t < SW; ++t) {
        double w = o.rv[t];
        w -= o.l[0][t] * o.yz[t];
        w -= o.l[1][t] * o.yy[t];
        w -= o.l[2][t] * v;
        d.y[SW * f + t * cnt + p] = w;
        v = w;
    }
}

// operands of one chunk's backward step: its forward values, the y+1 and z+1
// neighbours' results (plane P + 1: first chunk fp, cp chunks), the x+1
// result of slot SW - 1, u and the pivot inverses
struct BwdOps {
    double yv[SW], zy[SW], zz[SW], u[3][SW], di[SW], zx;
};

__device__ inline void bwd_load(const SRasDev &d, const ChunkIds &k, int64_t f, int64_t cnt, int64_t p, int64_t fp,
                                int64_t cp, BwdOps &o)
{
    const int64_t ns = SW * d.nitem;
    const bool live = p < cnt;
#pragma unroll
    for (int t = 0; t < SW; ++t) {
        const int64_t e = SW * f + t * cnt + p;
        o.yv[t] = live ? d.y[e] : 0.0;
        o.zy[t] = k.b >= 0 ? d.y[SW * fp + t * cp + k.b] : 0.0;
        o.zz[t] = k.c >= 0 ? d.y[SW * fp + t * cp + k.c] : 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) o.u[a][t] = live ? __builtin_nontemporal_load(d.u + a * ns + e) : 0.0;
        o.di[t] = live ? __builtin_nontemporal_load(d.dinv + e) : 0.0;
    }
    o.zx = k.a >= 0 ? d.y[SW * fp + k.a] : 0.0;
}

__device__ inline void bwd_solve(const SRasDev &d, double *zout, const ChunkIds &k, int64_t f, int64_t cnt,
                                 int64_t p, const BwdOps &o)
{
    if (p >= cnt) return;
    double v = o.zx;
#pragma unroll
    for (int t = SW - 1; t >= 0; --t) {
        double w = o.yv[t];
        w -= o.u[0][t] * v;
        w -= o.u[1][t] * o.zy[t];
        w -= o.u[2][t] * o.zz[t];
        w *= o.di[t];
        d.y[SW * f + t * cnt + p] = w;
        if ((k.m >> (OWN_SHIFT + t)) & 1) zout[k.r0 + t] = w;
        v = w;
    }
}

// forward y_c = r_c - sum_k l_ck y_k over the planes, then backward
// z_c = (y_c - sum_m u_cm z_m) / D_c in reverse; the owner of a cell writes z.
// A thread takes positions tid and tid + APPLY_T of every plane (and more on
// planes of over 2 APPLY_T chunks); their ids are read one plane ahead, and
// in the forward sweep the operands of both are loaded before either is
// solved, so a plane costs one round trip to memory.  The factors are
// streamed past the caches' retention (one slot of a plane's chunks is one
// contiguous row); r and z, which a thread reads and writes 8 bytes at a time
// along its chunk, and the sweeps' values, which the next plane reads, go
// through the caches (streaming r and z as well doubled the traffic).
__global__ __launch_bounds__(APPLY_T) void k_sras_apply(SRasDev d, const double *__restrict__ rin,
                                                        double *__restrict__ zout)
{
    const int s = blockIdx.x, np = d.pl_cnt[s], tid = threadIdx.x;
    const int64_t *pl = d.pl + d.pl_off[s];
    if (np <= 0) return;
    ChunkIds n0 = chunk_ids(d, d.nlo, pl[0], pl[1] - pl[0], tid);
    ChunkIds n1 = chunk_ids(d, d.nlo, pl[0], pl[1] - pl[0], tid + APPLY_T);
    for (int P = 0; P < np; ++P) {
        const int64_t f = pl[P], cnt = pl[P + 1] - f;
        const int64_t fm = P > 0 ? pl[P - 1] : f, cm = f - fm;
        const ChunkIds k0 = n0, k1 = n1;
        if (P + 1 < np) {
            const int64_t fn = pl[P + 1], cn = pl[P + 2] - fn;
            n0 = chunk_ids(d, d.nlo, fn, cn, tid);
            n1 = chunk_ids(d, d.nlo, fn, cn, tid + APPLY_T);
        }
        FwdOps o0, o1;
        fwd_load(d, rin, k0, f, cnt, tid, fm, cm, o0);
        fwd_load(d, rin, k1, f, cnt, tid + APPLY_T, fm, cm, o1);
        fwd_solve(d, f, cnt, tid, o0);
        fwd_solve(d, f, cnt, tid + APPLY_T, o1);
        for (int64_t p = tid + 2 * APPLY_T; p < cnt; p += APPLY_T) {
            const ChunkIds k = chunk_ids(d, d.nlo, f, cnt, p);
            fwd_load(d, rin, k, f, cnt, p, fm, cm, o0);
            fwd_solve(d, f, cnt, p, o0);
        }
        __syncthreads();
    }
    n0 = chunk_ids(d, d.nhi, pl[np - 1], pl[np] - pl[np - 1], tid);
    n1 = chunk_ids(d, d.nhi, pl[np - 1], pl[np] - pl[np - 1], tid + APPLY_T);
    for (int P = np - 1; P >= 0; --P) {
        const int64_t f = pl[P], cnt = pl[P + 1] - f;
        const int64_t fp = pl[P + 1], cp = P + 1 < np ? pl[P + 2] - fp : 0;
        const ChunkIds k0 = n0, k1 = n1;
        if (P > 0) {
            const int64_t fn = pl[P - 1], cn = f - fn;
            n0 = chunk_ids(d, d.nhi, fn, cn, tid);
            n1 = chunk_ids(d, d.nhi, fn, cn, tid + APPLY_T);
        }
        BwdOps o;                      // one chunk at a time: two would not fit the registers
        bwd_load(d, k0, f, cnt, tid, fp, cp, o);
        bwd_solve(d, zout, k0, f, cnt, tid, o);
        if (tid + APPLY_T < cnt) {
            bwd_load(d, k1, f, cnt, tid + APPLY_T, fp, cp, o);
            bwd_solve(d, zout, k1, f, cnt, tid + APPLY_T, o);
        }
        for (int64_t p = tid + 2 * APPLY_T; p < cnt; p += APPLY_T) {
            const ChunkIds k = chunk_ids(d, d.nhi, f, cnt, p);
            bwd_load(d, k, f, cnt, p, fp, cp, o);
            bwd_solve(d, zout, k, f, cnt, p, o);
        }
        __syncthreads();
    }
}

int64_t box_start(int64_t b, int64_t len, int64_t p)
{
    const int64_t base = len / p, rem = len % p;
    return b * base + std::min(b, rem);
}

struct SRas final : PcImpl {
    rsv_matrix *M = nullptr;
    rsv_ctx *c = nullptr;
    int nsub = 0;
    int64_t nitem = 0, ncell = 0, tplanes = 0;   // chunks, Omega_s cells, plane table entries
    std::vector<void *> mem;
    SRasDev d{};

    ~SRas() override
    {
        if (c) (void)hipStreamSynchronize(c->stream);
        for (void *p : mem) dev_free(p);
    }
    // per chunk: row, mask, 3 + 3 neighbour positions (32 B); per slot: 3 + 3
    // coefficients, the pivot inverse and the working value (64 B)
    int64_t bytes() const override { return nitem * (32 + SW * 64) + tplanes * 8 + nsub * 8; }
    // per Omega_s cell: 3 + 3 coefficients and the pivot inverse (56 B), r in,
    // y out, y in (24 B); z out once per grid cell; per chunk its 32 B
    int64_t apply_bytes() const override
    {
        const Geo &G = M->g->geo;
        return ncell * 80 + (int64_t)G.nx * G.ny * G.nz * 8 + nitem * 32;
    }

    template <class T> rsv_status alloc(T **p, size_t n)
    {
        rsv_status s = dev_alloc(c, (void **)p, n * sizeof(T));
        if (s == RSV_OK) mem.push_back(*p);
        return s;
    }

    rsv_status apply(const double *r, double *z) override
    {
        ProfScope ps(c, RSV_K_RAS);
        hipLaunchKernelGGL(k_sras_apply, dim3(nsub), dim3(APPLY_T), 0, c->stream, d, r, z);
        RSV_LAUNCH(c);
        return RSV_OK;
    }

    rsv_status setup(int px, int py, int pz, int ov, int64_t *bad_cell)
    {
        const Geo &G = M->g->geo;
        const int64_t nx = G.nx, ny = G.ny, nz = G.nz;
        if (nx * ny * nz >= ((int64_t)1 << 31)) return set_err(c, RSV_ERR_ARG, "scalar RAS: more than 2^31 cells");
        nsub = px * py * pz;
        // per subdomain: its box, extended box, chunk count and first chunk
        struct Box { int64_t x0, x1, y0, y1, z0, z1, ex0, ex1, ey0, ey1, ez0, ez1, nc, count, first; int nplane; };
        std::vector<Box> B(nsub);
        for (int s = 0; s < nsub; ++s) {
            Box &b = B[s];
            const int sx = s % px, sy = (s / px) % py, sz = s / (px * py);
            b.x0 = box_start(sx, nx, px); b.x1 = box_start(sx + 1, nx, px);
            b.y0 = box_start(sy, ny, py); b.y1 = box_start(sy + 1, ny, py);
            b.z0 = box_start(sz, nz, pz); b.z1 = box_start(sz + 1, nz, pz);
            b.ex0 = std::max<int64_t>(0, b.x0 - ov); b.ex1 = std::min<int64_t>(nx, b.x1 + ov);
            b.ey0 = std::max<int64_t>(0, b.y0 - ov); b.ey1 = std::min<int64_t>(ny, b.y1 + ov);
            b.ez0 = std::max<int64_t>(0, b.z0 - ov); b.ez1 = std::min<int64_t>(nz, b.z1 + ov);
            b.nc = (b.ex1 - b.ex0 + SW - 1) / SW;
            b.nplane = (int)(b.nc + (b.ey1 - b.ey0) + (b.ez1 - b.ez0) - 2);
        }
        auto dist = [](int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo - v : (v >= hi ? v - hi + 1 : 0); };
        // the cells of grid row (j, k) inside Omega_s: one x-interval [lo, hi)
        auto row_range = [&](const Box &b, int64_t j, int64_t k, int64_t &lo, int64_t &hi) {
            const int64_t rest = dist(j, b.y0, b.y1) + dist(k, b.z0, b.z1);
            if (rest > ov) return false;
            lo = std::max(b.ex0, b.x0 - (ov - rest));
            hi = std::min(b.ex1, b.x1 + (ov - rest));
            return hi > lo;
        };
        int64_t total = 0, cells = 0;
        tplanes = 0;
        for (int s = 0; s < nsub; ++s) {
            Box &b = B[s];
            int64_t cnt = 0, lo, hi;
            for (int64_t k = b.ez0; k < b.ez1; ++k)
                for (int64_t j = b.ey0; j < b.ey1; ++j)
                    if (row_range(b, j, k, lo, hi)) {
                        cnt += (hi - 1 - b.ex0) / SW - (lo - b.ex0) / SW + 1;
                        cells += hi - lo;
                    }
            b.count = cnt;
            b.first = total;
            total += cnt;
            tplanes += b.nplane + 1;
        }
        nitem = total;
        ncell = cells;
        std::vector<int32_t> row0(total), mask(total), nlo(3 * total), nhi(3 * total);
        std::vector<int64_t> pl(tplanes);
        std::vector<int32_t> pl_off(nsub), pl_cnt(nsub);
        {
            int64_t off = 0;
            for (int s = 0; s < nsub; ++s) {
                pl_off[s] = (int32_t)off;
                pl_cnt[s] = B[s].nplane;
                off += B[s].nplane + 1;
            }
        }
        auto build = [&](int s) {
            const Box &b = B[s];
            const int64_t NC = b.nc, EY = b.ey1 - b.ey0, EZ = b.ez1 - b.ez0;
            const int NP = b.nplane;
            std::vector<int64_t> start(NP + 1, 0);
            int64_t lo, hi;
            for (int64_t k = 0; k < EZ; ++k)
                for (int64_t j = 0; j < EY; ++j)
                    if (row_range(b, b.ey0 + j, b.ez0 + k, lo, hi))
                        for (int64_t cc = (lo - b.ex0) / SW; cc <= (hi - 1 - b.ex0) / SW; ++cc) start[cc + j + k + 1]++;
            for (int P = 0; P < NP; ++P) start[P + 1] += start[P];
            int64_t *plp = pl.data() + pl_off[s];
            for (int P = 0; P <= NP; ++P) plp[P] = b.first + start[P];
            std::vector<int32_t> pos((size_t)(NC * EY * EZ), -1);
            std::vector<int64_t> fill(NP, 0);
            for (int64_t k = 0; k < EZ; ++k)                  // (k, j, c) order inside every plane
                for (int64_t j = 0; j < EY; ++j) {
                    if (!row_range(b, b.ey0 + j, b.ez0 + k, lo, hi)) continue;
                    const int64_t gj = b.ey0 + j, gk = b.ez0 + k;
                    const bool own_row = gj >= b.y0 && gj < b.y1 && gk >= b.z0 && gk < b.z1;
                    for (int64_t cc = (lo - b.ex0) / SW; cc <= (hi - 1 - b.ex0) / SW; ++cc) {
                        const int64_t P = cc + j + k, p = fill[P]++;
                        pos[(k * EY + j) * NC + cc] = (int32_t)p;
                        const int64_t q = b.first + start[P] + p;
                        const int64_t x = b.ex0 + cc * SW;
                        row0[q] = (int32_t)row_of(G, (int)x, (int)gj, (int)gk);
                        int mk = 0;
                        for (int t = 0; t < SW; ++t) {
                            const int64_t i = x + t;
                            if (i < lo || i >= hi) continue;
                            mk |= 1 << t;
                            if (own_row && i >= b.x0 && i < b.x1) mk |= 1 << (OWN_SHIFT + t);
                        }
                        mask[q] = mk;
                    }
                }
            auto at = [&](int64_t cc, int64_t j, int64_t k) -> int32_t {
                if (cc < 0 || cc >= NC || j < 0 || j >= EY || k < 0 || k >= EZ) return -1;
                return pos[(k * EY + j) * NC + cc];
            };
            for (int64_t k = 0; k < EZ; ++k)
                for (int64_t j = 0; j < EY; ++j)
                    for (int64_t cc = 0; cc < NC; ++cc) {
                        const int32_t p = at(cc, j, k);
                        if (p < 0) continue;
                        const int64_t q = b.first + start[cc + j + k] + p;
                        nlo[0 * total + q] = at(cc, j, k - 1);
                        nlo[1 * total + q] = at(cc, j - 1, k);
                        nlo[2 * total + q] = at(cc - 1, j, k);
                        nhi[0 * total + q] = at(cc + 1, j, k);
                        nhi[1 * total + q] = at(cc, j + 1, k);
                        nhi[2 * total + q] = at(cc, j, k + 1);
                    }
        };
        {
            const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
            std::vector<std::thread> th;
            for (int t = 0; t < nth; ++t)
                th.emplace_back([&, t] { for (int s = t; s < nsub; s += nth) build(s); });
            for (auto &x : th) x.join();
        }
        int32_t *drow0, *dmask, *dlo, *dhi, *dploff, *dplcnt;
        int64_t *dpl;
        double *dl, *du, *ddinv, *dy;
        const size_t nslot = (size_t)SW * total;
        rsv_status st = alloc(&drow0, (size_t)total);
        if (st == RSV_OK) st = alloc(&dmask, (size_t)total);
        if (st == RSV_OK) st = alloc(&dlo, (size_t)3 * total);
        if (st == RSV_OK) st = alloc(&dhi, (size_t)3 * total);
        if (st == RSV_OK) st = alloc(&dl, 3 * nslot);
        if (st == RSV_OK) st = alloc(&du, 3 * nslot);
        if (st == RSV_OK) st = alloc(&ddinv, nslot);
        if (st == RSV_OK) st = alloc(&dy, nslot);
        if (st == RSV_OK) st = alloc(&dpl, (size_t)tplanes);
        if (st == RSV_OK) st = alloc(&dploff, (size_t)nsub);
        if (st == RSV_OK) st = alloc(&dplcnt, (size_t)nsub);
        if (st != RSV_OK) return st;
        RSV_HIP(c, hipMemcpyAsync(drow0, row0.data(), total * 4, hipMemcpyHostToDevice, c->stream));
        RSV_HIP(c, hipMemcpyAsync(dmask, mask.data(), total * 4, hipMemcpyHostToDevice, c->stream));
        RSV_HIP(c, hipMemcpyAsync(dlo, nlo.data(), 3 * total * 4, hipMemcpyHostToDevice, c->stream));
        RSV_HIP(c, hipMemcpyAsync(dhi, nhi.data(), 3 * total * 4, hipMemcpyHostToDevice, c->stream));
        RSV_HIP(c, hipMemcpyAsync(dpl, pl.data(), tplanes * 8, hipMemcpyHostToDevice, c->stream));
        RSV_HIP(c, hipMemcpyAsync(dploff, pl_off.data(), nsub * 4, hipMemcpyHostToDevice, c->stream));
        RSV_HIP(c, hipMemcpyAsync(dplcnt, pl_cnt.data(), nsub * 4, hipMemcpyHostToDevice, c->stream));
        d = SRasDev{total, drow0, dmask, dlo, dhi, dl, du, ddinv, dy, dpl, dploff, dplcnt};
        rsv_status fs = flags_reset(c);   // synchronises: the host arrays may be released after it
        if (fs != RSV_OK) return fs;
        {
            ProfScope ps(c, RSV_K_FACTOR);
            hipLaunchKernelGGL(k_sras_factor, dim3(nsub), dim3(RAS_T), 0, c->stream, G, M->d_coef, d, c->d_flags);
        }
        RSV_LAUNCH(c);
        return flags_check(c, bad_cell);
    }
};

}  // namespace

rsv_status launch_sspmv(rsv_ctx *c, const Geo &g, const double *coef, int mode, const double *x, double *y,
                        const double *aux, double alpha, double beta, int k0)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int nb = (int)((n + SB - 1) / SB);
    if (mode >= SPMV_RESID) {
        rsv_status s = partials_reserve(c, (int64_t)nb * 2);
        if (s != RSV_OK) return s;
    }
    double *P = c->d_partials;
    const int tok = prof_begin(c, RSV_K_SPMV);
    const dim3 grid(nb), blk(SB);
    switch (mode) {
    case SPMV_Y: hipLaunchKernelGGL(k_sspmv<SPMV_Y>, grid, blk, 0, c->stream, g, coef, x, y, aux, alpha, beta, P); break;
    case SPMV_AXPBY: hipLaunchKernelGGL(k_sspmv<SPMV_AXPBY>, grid, blk, 0, c->stream, g, coef, x, y, aux, alpha, beta, P); break;
    case SPMV_RESID: hipLaunchKernelGGL(k_sspmv<SPMV_RESID>, grid, blk, 0, c->stream, g, coef, x, y, aux, alpha, beta, P); break;
    case SPMV_NORM: hipLaunchKernelGGL(k_sspmv<SPMV_NORM>, grid, blk, 0, c->stream, g, coef, x, y, aux, alpha, beta, P); break;
    case SPMV_DOT1: hipLaunchKernelGGL(k_sspmv<SPMV_DOT1>, grid, blk, 0, c->stream, g, coef, x, y, aux, alpha, beta, P); break;
    case SPMV_DOT2: hipLaunchKernelGGL(k_sspmv<SPMV_DOT2>, grid, blk, 0, c->stream, g, coef, x, y, aux, alpha, beta, P); break;
    default: return set_err(c, RSV_ERR_ARG, "bad spmv mode");
    }
    prof_end(c, tok);
    RSV_LAUNCH(c);
    if (mode >= SPMV_RESID) return launch_reduce(c, nb, mode == SPMV_DOT2 ? 2 : 1, k0);
    return RSV_OK;
}

rsv_status mat_spmv(rsv_matrix *M, int mode, const double *x, double *y, const double *aux, double alpha,
                    double beta, int k0)
{
    if (M->bs == 1) return launch_sspmv(M->g->ctx, M->g->geo, M->d_coef, mode, x, y, aux, alpha, beta, k0);
    return launch_spmv(M->g->ctx, M->g->geo, M->d_A, mode, x, y, aux, alpha, beta, k0);
}

rsv_status mat_in(rsv_matrix *M, const double *nat, double *v)
{
    if (M->bs == 1) return launch_copy(M->g->ctx, M->nv, nat, v);
    return launch_nat_to_tl(M->g->ctx, M->g->geo, nat, v);
}

rsv_status mat_out(rsv_matrix *M, const double *v, double *nat, double alpha, double beta)
{
    if (M->bs == 1) return launch_axpby(M->g->ctx, M->nv, alpha, v, beta, nat);
    return launch_tl_to_nat(M->g->ctx, M->g->geo, v, nat, alpha, beta);
}

rsv_status sras_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell)
{
    rsv_ctx *c = A->g->ctx;
    const Geo &G = A->g->geo;
    int px = 1, py = 1, pz = 1, ov = 0;      // BILU0 of a scalar matrix: one subdomain, no overlap
    if (p->type == RSV_PC_RAS) {
        px = p->ras_px; py = p->ras_py; pz = p->ras_pz; ov = p->ras_overlap;
        if (px < 1 || py < 1 || pz < 1 || px > G.nx || py > G.ny || pz > G.nz || ov < 0)
            return set_err(c, RSV_ERR_ARG, "bad RAS subdomain counts or overlap");
    }
    if (p->precision != RSV_FP64) return set_err(c, RSV_ERR_ARG, "scalar systems have FP64 preconditioners only");
    SRas *R = new (std::nothrow) SRas();
    if (!R) return set_err(c, RSV_ERR_OOM, "scalar RAS");
    R->M = A;
    R->c = c;
    rsv_status s = R->setup(px, py, pz, ov, bad_cell);
    if (s != RSV_OK) {
        delete R;
        return s;
    }
    *out = R;
    return RSV_OK;
}

extern "C" {

rsv_status rsv_matrix_assemble_scalar(rsv_grid *g, const double *coef, int32_t where, rsv_matrix **out)
{
    if (!g || !coef || !out) return set_err(g ? g->ctx : nullptr, RSV_ERR_ARG, "NULL argument");
    *out = nullptr;
    rsv_ctx *c = g->ctx;
    rsv_matrix *M = new (std::nothrow) rsv_matrix();
    if (!M) return set_err(c, RSV_ERR_OOM, "matrix");
    M->g = g;
    M->bs = 1;
    M->nv = g->ncell;
    rsv_status s = dev_alloc(c, (void **)&M->d_coef, (size_t)g->ncell * 7 * sizeof(double));
    if (s == RSV_OK) {
        M->bytes = g->ncell * 7 * (int64_t)sizeof(double);
        s = scalar_assemble_values(M, coef, where);
    }
    if (s != RSV_OK) {
        rsv_matrix_destroy(M);
        return s;
    }
    *out = M;
    return RSV_OK;
}

}  // extern "C"

rsv_status scalar_assemble_values(rsv_matrix *M, const double *coef, int32_t where)
{
    rsv_grid *g = M->g;
    rsv_ctx *c = g->ctx;
    const size_t bytes = (size_t)g->ncell * 7 * sizeof(double);
    const double *src = coef;
    double *stage = nullptr;
    if (where == RSV_MEM_HOST) {
        rsv_status s = dev_alloc(c, (void **)&stage, bytes);
        if (s != RSV_OK) return s;
        hipError_t e = hipMemcpyAsync(stage, coef, bytes, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) {
            dev_free(stage);
            return set_err(c, RSV_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
        }
        src = stage;
    } else if (where != RSV_MEM_DEVICE) {
        return set_err(c, RSV_ERR_ARG, "bad memory kind");
    }
    rsv_status s = flags_reset(c);
    if (s == RSV_OK) {
        hipLaunchKernelGGL(k_sassemble, dim3((unsigned)((g->ncell + SB - 1) / SB)), dim3(SB), 0, c->stream, g->geo, src,
                           M->d_coef, c->d_flags);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) s = set_err(c, RSV_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    if (s == RSV_OK) s = flags_check(c, nullptr);
    if (stage) dev_free(stage);
    return s;
}
